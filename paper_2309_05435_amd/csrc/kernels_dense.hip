// Dense FP64 kernels for the spatial blocks of the block-tridiagonal chains:
//   - grouped GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4f64);
//   - in-place inversion of SPD blocks by the block Gauss-Jordan sweep:
//     register-resident for order <= 128, rank-128 outer steps on the
//     matrix cores above;
//   - products of the restricted 13-point stencil Q_R with dense blocks.
// Dense blocks are column-major, padded to multiples of 64 with identity on
// the padded diagonal.
#include <climits>

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
// In MFMA step s lane group g = l/16 contributes k = 4g + s.  LDS layouts,
// chosen so that the stores of a tile and the fragment reads are free of bank
// conflicts:
//   - A^T operand, B operand (k contiguous in memory): row m (or column n) of
//     the tile holds its 16 k values, rows 18 apart; a lane reads its four k
//     of a row with one 32-byte access;
//   - A operand (m contiguous in memory): k row of the tile holds its 128 m
//     values, rows 132 apart; a lane reads its four k with 8-byte accesses.
//     Each global load instruction covers two consecutive m per lane over 16
//     lanes (256 contiguous bytes), stored the same way.
// The transposes and whether the tile lies wholly inside C are template
// parameters of the K loop (a uniform branch per workgroup picks the
// instance), so the interior tiles run without bounds checks.
// ---------------------------------------------------------------------------
namespace {
constexpr int GBM = 128, GBN = 128, GBK = 16, GLDS = GBK + 2;
constexpr int GAM = GBM + 4;  // k-row stride of the m-major A tile
constexpr int GAS = GBM * GLDS > GBK * GAM ? GBM * GLDS : GBK * GAM;

// Each thread moves 8 doubles of the A tile and 8 of the B tile per K step.
struct TileRegs {
  double2 v[4];
};

template <int TA, bool FULL>
__device__ __forceinline__ void load_a(const GemmTask& tk, int m0, int k0, int tid, TileRegs& r) {
  if (!TA) {  // k row tid / 16; m pairs at 2 (tid % 16) + 32 j
    const int kk = tid >> 4, mb = 2 * (tid & 15);
    const gptr<const double> src = G(tk.A) + (size_t)(k0 + kk) * tk.lda + m0 + mb;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = m0 + mb + 32 * j;
      if (FULL || c + 1 < tk.M) r.v[j] = ldg2(src + 32 * j);
      else r.v[j] = double2{c < tk.M ? src[32 * j] : 0.0, 0.0};
    }
  } else {  // A^T stored column-major: 8 consecutive k of one row m
    const int mm = tid >> 1, kk = (tid & 1) * 8, gm = m0 + mm;
    const gptr<const double> src = G(tk.A) + (size_t)gm * tk.lda + k0 + kk;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      r.v[j] = (FULL || gm < tk.M) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
  }
}

template <int TA>
__device__ __forceinline__ void store_a(int tid, const TileRegs& r, double* As) {
  if (!TA) {
    const int kk = tid >> 4, mb = 2 * (tid & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2*)&As[kk * GAM + mb + 32 * j] = r.v[j];
  } else {
    const int mm = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2*)&As[mm * GLDS + kk + 2 * j] = r.v[j];
  }
}

template <int TB, bool FULL>
__device__ __forceinline__ void load_b(const GemmTask& tk, int n0, int k0, int tid, TileRegs& r) {
  if (!TB) {  // column-major B: 8 consecutive k of one column n
    const int nn = tid >> 1, kk = (tid & 1) * 8, gn = n0 + nn;
    const gptr<const double> src = G(tk.B) + (size_t)gn * tk.ldb + k0 + kk;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      r.v[j] = (FULL || gn < tk.N) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
  } else {  // B^T stored column-major: 8 consecutive n of one row k
    const int kk = tid >> 4, nn = (tid & 15) * 8, gn = n0 + nn;
    const gptr<const double> src = G(tk.B) + (size_t)(k0 + kk) * tk.ldb + gn;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = gn + 2 * j;
      if (FULL || c + 1 < tk.N) r.v[j] = ldg2(src + 2 * j);
      else r.v[j] = double2{c < tk.N ? src[2 * j] : 0.0, 0.0};
    }
  }
}

template <int TB>
__device__ __forceinline__ void store_b(int tid, const TileRegs& r, double* Bs) {
  if (!TB) {
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

// The K loop of one tile.  The A/B tiles of steps k + 1 and k + 2 are in
// registers (loads in flight) while the matrix cores consume step k from LDS;
// the LDS tiles are double-buffered, so one barrier per K step separates the
// stores of step k + 1 from the reads of step k.  Each step's fragments are
// read in two halves (k = 4g + {0, 1}, then 4g + {2, 3}), which keeps the
// second prefetch within the register budget; the products are accumulated
// in the same order as with whole fragments.
template <int TA, int TB, bool FULL>
__device__ __forceinline__ void gemm_tile(const GemmTask& tk, int m0, int n0, v4d (&acc)[4][4],
                                          double* As0, double* As1, double* Bs0, double* Bs1) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int l16 = lane & 15, g = lane >> 4;
  const int nk = tk.K / GBK;
  TileRegs ga[2], gb[2];
  load_a<TA, FULL>(tk, m0, 0, tid, ga[0]);
  load_b<TB, FULL>(tk, n0, 0, tid, gb[0]);
  if (nk > 1) {
    load_a<TA, FULL>(tk, m0, GBK, tid, ga[1]);
    load_b<TB, FULL>(tk, n0, GBK, tid, gb[1]);
  }
  store_a<TA>(tid, ga[0], As0);
  store_b<TB>(tid, gb[0], Bs0);
  __syncthreads();
  auto half = [&](const double* Ac, const double* Bc, int h) {
    double a[4][2], bb[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!TA) {
#pragma unroll
        for (int s = 0; s < 2; ++s) a[i][s] = Ac[(4 * g + 2 * h + s) * GAM + wm + i * 16 + l16];
      } else {
        const double2 x = *(const double2*)&Ac[(wm + i * 16 + l16) * GLDS + 4 * g + 2 * h];
        a[i][0] = x.x;
        a[i][1] = x.y;
      }
      const double2 y = *(const double2*)&Bc[(wn + i * 16 + l16) * GLDS + 4 * g + 2 * h];
      bb[i][0] = y.x;
      bb[i][1] = y.y;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(bb[j][s], a[i][s], acc[i][j]);
  };
  // step k (P = k & 1): LDS buffer P holds step k, registers [P] are free for
  // step k + 2, registers [1 - P] hold step k + 1; buffer 1 - P was last read
  // before the previous barrier
#define RBMC_GEMM_STEP(P)                                                          \
  {                                                                                \
    double* Ac = P ? As1 : As0;                                                    \
    double* Bc = P ? Bs1 : Bs0;                                                    \
    if (k + 2 < nk) {                                                              \
      load_a<TA, FULL>(tk, m0, (k + 2) * GBK, tid, ga[P]);                         \
      load_b<TB, FULL>(tk, n0, (k + 2) * GBK, tid, gb[P]);                         \
    }                                                                              \
    half(Ac, Bc, 0);                                                               \
    half(Ac, Bc, 1);                                                               \
    if (k + 1 < nk) {                                                              \
      store_a<TA>(tid, ga[1 - P], P ? As0 : As1);                                  \
      store_b<TB>(tid, gb[1 - P], P ? Bs0 : Bs1);                                  \
    }                                                                              \
    __syncthreads();                                                               \
    ++k;                                                                           \
  }
  int k = 0;
  while (k < nk) {
    RBMC_GEMM_STEP(0)
    if (k < nk) RBMC_GEMM_STEP(1)
  }
#undef RBMC_GEMM_STEP
}
}  // namespace

int gemm_task_tiles(int M, int N, int lower, int ts) {
  const int tm = (M + ts - 1) / ts, tn = (N + ts - 1) / ts;
  return lower ? tm * (tm + 1) / 2 : tm * tn;
}

// Workgroups are dispatched round-robin over the 8 XCDs; the logical tile of
// a workgroup is chosen so that each XCD walks a contiguous range of tiles
// (neighbouring tiles share A row panels in its L2).  K is a multiple of 16.
// TAG only names the instantiation (1: the spectral transforms), so kernel
// traces and counters separate the two uses; the code is the same.
template <int TAG>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(const GemmTask* __restrict__ tasks,
                                                     int n_tasks, int total_tiles, int per_xcd) {
  __shared__ double As[2][GAS];
  __shared__ double Bs[2][GBN * GLDS];
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
  const bool full = m0 + GBM <= tk.M && n0 + GBN <= tk.N;
  const int tt = tk.transA * 2 + tk.transB;
#define RBMC_GEMM_TILE(TA_, TB_)                                                       \
  (full ? gemm_tile<TA_, TB_, true>(tk, m0, n0, acc, As[0], As[1], Bs[0], Bs[1])      \
        : gemm_tile<TA_, TB_, false>(tk, m0, n0, acc, As[0], As[1], Bs[0], Bs[1]))
  if (tt == 0) RBMC_GEMM_TILE(0, 0);
  else if (tt == 1) RBMC_GEMM_TILE(0, 1);
  else if (tt == 2) RBMC_GEMM_TILE(1, 0);
  else RBMC_GEMM_TILE(1, 1);
#undef RBMC_GEMM_TILE
  // ---- epilogue: C = alpha acc + beta Cin.  The products were formed as
  // (B^T A^T) tiles, so register r of lane l holds C[16 i + l%16][16 j + l/16
  // + 4 r]: 16 consecutive rows of a column per lane group (128-byte segments).
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + wm + i * 16 + l16;
    if (gm >= tk.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn + j * 16 + g + 4 * r;
        if (gn >= tk.N) continue;
        double v = tk.alpha * acc[i][j][r];
        if (tk.beta != 0.0) v += tk.beta * G(tk.Cin)[(size_t)gn * tk.ldcin + gm];
        G(tk.C)[(size_t)gn * tk.ldc + gm] = v;
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
// register i of lane l holds C[4 (l/16) + i][l%16].  As in the FP64 kernels
// the tile is formed transposed (B^T A^T), so the stores run down columns.
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
    const gptr<const double> src = G(tk.A) + (size_t)(k0 + kk) * tk.lda + gm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gm + 2 * j;
      if (c + 1 < tk.M) r.v[j] = ldg2(src + 2 * j);
      else r.v[j] = double2{c < tk.M ? src[2 * j] : 0.0, 0.0};
    }
  } else {  // 4 consecutive k of row m
    const int gm = m0 + (tid >> 2), kk = (tid & 3) * 4;
    const gptr<const double> src = G(tk.A) + (size_t)gm * tk.lda + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gm < tk.M) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
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
    const gptr<const double> src = G(tk.B) + (size_t)gn * tk.ldb + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gn < tk.N) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
  } else {  // 4 consecutive n of row k
    const int kk = tid >> 5, gn = n0 + (tid & 31) * 4;
    const gptr<const double> src = G(tk.B) + (size_t)(k0 + kk) * tk.ldb + gn;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gn + 2 * j;
      if (c + 1 < tk.N) r.v[j] = ldg2(src + 2 * j);
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
  __shared__ float As[2][GBM * XLD];
  __shared__ float Bs[2][GBN * XLD];
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
  xstore_a(tk, tid, ra, As[0]);
  xstore_b(tk, tid, rb, Bs[0]);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < tk.K; k0 += GBK) {
    const bool more = k0 + GBK < tk.K;
    if (more) {
      xload_a(tk, m0, k0 + GBK, tid, ra);
      xload_b(tk, n0, k0 + GBK, tid, rb);
    }
    float4 a[4], bb[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const float4*)&As[buf][(wm + i * 16 + l16) * XLD + 4 * g];
#pragma unroll
    for (int j = 0; j < 2; ++j) bb[j] = *(const float4*)&Bs[buf][(wn + j * 16 + l16) * XLD + 4 * g];
    v4f c32[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) c32[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[j].x, a[i].x, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[j].y, a[i].y, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[j].z, a[i].z, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[j].w, a[i].w, c32[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c32[i][j][r];
    if (more) {  // the other buffer was last read before the previous barrier
      xstore_a(tk, tid, ra, As[buf ^ 1]);
      xstore_b(tk, tid, rb, Bs[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  // transposed tile products: register r of lane l holds C[16 i + l%16][16 j + 4 (l/16) + r]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + wm + i * 16 + l16;
    if (gm >= tk.M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn + j * 16 + 4 * g + r;
        if (gn >= tk.N) continue;
        double v = tk.alpha * acc[i][j][r];
        if (tk.beta != 0.0) v += tk.beta * G(tk.Cin)[(size_t)gn * tk.ldcin + gm];
        G(tk.C)[(size_t)gn * tk.ldc + gm] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// Grouped FP64 GEMM with 64 x 64 tiles (four waves of 32 x 32), for launches
// with too few 128 x 128 tiles to fill the device: a small working set per
// workgroup lets several workgroups share a CU and hide memory latency.
// Same task semantics (lower mode and skip ranges on 64-tiles).
// ---------------------------------------------------------------------------
namespace {
constexpr int SB = 64;

__device__ inline void sload_a(const GemmTask& tk, int m0, int k0, int tid, XRegs& r) {
  if (!tk.transA) {  // 4 consecutive rows of column k
    const int kk = tid >> 4, gm = m0 + (tid & 15) * 4;
    const gptr<const double> src = G(tk.A) + (size_t)(k0 + kk) * tk.lda + gm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gm + 2 * j;
      if (c + 1 < tk.M) r.v[j] = ldg2(src + 2 * j);
      else r.v[j] = double2{c < tk.M ? src[2 * j] : 0.0, 0.0};
    }
  } else {  // 4 consecutive k of row m
    const int gm = m0 + (tid >> 2), kk = (tid & 3) * 4;
    const gptr<const double> src = G(tk.A) + (size_t)gm * tk.lda + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gm < tk.M) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
  }
}

__device__ inline void sstore_a(const GemmTask& tk, int tid, const XRegs& r, double* As) {
  if (!tk.transA) {
    const int kk = tid >> 4, mm = (tid & 15) * 4;
    As[(mm + 0) * GLDS + kk] = r.v[0].x;
    As[(mm + 1) * GLDS + kk] = r.v[0].y;
    As[(mm + 2) * GLDS + kk] = r.v[1].x;
    As[(mm + 3) * GLDS + kk] = r.v[1].y;
  } else {
    const int mm = tid >> 2, kk = (tid & 3) * 4;
    *(double2*)&As[mm * GLDS + kk] = r.v[0];
    *(double2*)&As[mm * GLDS + kk + 2] = r.v[1];
  }
}

__device__ inline void sload_b(const GemmTask& tk, int n0, int k0, int tid, XRegs& r) {
  if (!tk.transB) {  // 4 consecutive k of column n
    const int gn = n0 + (tid >> 2), kk = (tid & 3) * 4;
    const gptr<const double> src = G(tk.B) + (size_t)gn * tk.ldb + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gn < tk.N) ? ldg2(src + 2 * j) : double2{0.0, 0.0};
  } else {  // 4 consecutive n of row k
    const int kk = tid >> 4, gn = n0 + (tid & 15) * 4;
    const gptr<const double> src = G(tk.B) + (size_t)(k0 + kk) * tk.ldb + gn;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gn + 2 * j;
      if (c + 1 < tk.N) r.v[j] = ldg2(src + 2 * j);
      else r.v[j] = double2{c < tk.N ? src[2 * j] : 0.0, 0.0};
    }
  }
}

__device__ inline void sstore_b(const GemmTask& tk, int tid, const XRegs& r, double* Bs) {
  if (!tk.transB) {
    const int nn = tid >> 2, kk = (tid & 3) * 4;
    *(double2*)&Bs[nn * GLDS + kk] = r.v[0];
    *(double2*)&Bs[nn * GLDS + kk + 2] = r.v[1];
  } else {
    const int kk = tid >> 4, nn = (tid & 15) * 4;
    Bs[(nn + 0) * GLDS + kk] = r.v[0].x;
    Bs[(nn + 1) * GLDS + kk] = r.v[0].y;
    Bs[(nn + 2) * GLDS + kk] = r.v[1].x;
    Bs[(nn + 3) * GLDS + kk] = r.v[1].y;
  }
}
}  // namespace

__global__ __launch_bounds__(256) void k_gemm_f64s(const GemmTask* __restrict__ tasks,
                                                   int n_tasks, int total_tiles, int per_xcd) {
  __shared__ double As[2][SB * GLDS];
  __shared__ double Bs[2][SB * GLDS];
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
  const int m0 = tm * SB, n0 = tn * SB;
  if (tk.skip1 > tk.skip0) {
    const bool rows_hit = m0 < tk.skip1 && m0 + SB > tk.skip0;
    const bool cols_hit = n0 < tk.skip1 && n0 + SB > tk.skip0;
    if (rows_hit || cols_hit) return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int l16 = lane & 15, g = lane >> 4;

  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  XRegs ra, rb;
  sload_a(tk, m0, 0, tid, ra);
  sload_b(tk, n0, 0, tid, rb);
  sstore_a(tk, tid, ra, As[0]);
  sstore_b(tk, tid, rb, Bs[0]);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < tk.K; k0 += GBK) {
    const bool more = k0 + GBK < tk.K;
    if (more) {
      sload_a(tk, m0, k0 + GBK, tid, ra);
      sload_b(tk, n0, k0 + GBK, tid, rb);
    }
    double a[2][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double* pa = &As[buf][(wm + i * 16 + l16) * GLDS + 4 * g];
      double2 x0 = *(const double2*)pa, x1 = *(const double2*)(pa + 2);
      a[i][0] = x0.x; a[i][1] = x0.y; a[i][2] = x1.x; a[i][3] = x1.y;
      const double* pb = &Bs[buf][(wn + i * 16 + l16) * GLDS + 4 * g];
      double2 y0 = *(const double2*)pb, y1 = *(const double2*)(pb + 2);
      bb[i][0] = y0.x; bb[i][1] = y0.y; bb[i][2] = y1.x; bb[i][3] = y1.y;
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma64(bb[j][s2], a[i][s2], acc[i][j]);
    if (more) {  // the other buffer was last read before the previous barrier
      sstore_a(tk, tid, ra, As[buf ^ 1]);
      sstore_b(tk, tid, rb, Bs[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  // transposed tile products: register r of lane l holds C[16 i + l%16][16 j + l/16 + 4 r]
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int gm = m0 + wm + i * 16 + l16;
    if (gm >= tk.M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn + j * 16 + g + 4 * r;
        if (gn >= tk.N) continue;
        double v = tk.alpha * acc[i][j][r];
        if (tk.beta != 0.0) v += tk.beta * G(tk.Cin)[(size_t)gn * tk.ldcin + gm];
        G(tk.C)[(size_t)gn * tk.ldc + gm] = v;
      }
  }
}

void launch_gemm(const GemmTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s,
                 int kind, int tag) {
  if (total_tiles <= 0) return;
  const int per_xcd = (total_tiles + 7) / 8;
  if (kind == kGemmMixed)
    k_gemm_mx<<<per_xcd * 8, 512, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
  else if (kind == kGemmSmall)
    k_gemm_f64s<<<per_xcd * 8, 256, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
  else if (tag == 1)
    k_gemm_f64<1><<<per_xcd * 8, 256, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
  else
    k_gemm_f64<0><<<per_xcd * 8, 256, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
}

// ---------------------------------------------------------------------------
// SPD inversion by the block Gauss-Jordan sweep.  Sweeping pivot k of a
// symmetric M:
//   M_kk <- -1/M_kk,  M_ik <- M_ik / M_kk,  M_kj <- M_kj / M_kk,
//   M_ij <- M_ij - M_ik M_kj / M_kk   (i, j != k);
// after all pivots M holds -A^-1.  Pivots are Schur complements of an SPD
// matrix, hence positive.  Blocks of order <= 128 are swept entirely in
// registers by one workgroup; larger blocks take outer rank-128 steps whose
// updates run on the matrix cores (k_gj2_* and the grouped GEMM).
// ---------------------------------------------------------------------------
namespace {
constexpr int IB = 128;  // order of the register-resident sweep
constexpr int IT = 1024; // threads, 32 x 32, each owning a 4 x 4 block
}  // namespace

// One workgroup per task inverts P (order w <= 128, column-major, ld, full
// symmetric) in place.  Rows/columns w..127 are identity.  Thread
// (tr, tc) = (tid / 32, tid % 32) keeps rows 4 tr .. 4 tr + 3 x columns
// 4 tc .. 4 tc + 3 in registers.  Pivot p: the owners of row p and of column
// p publish them (and the pivot's owner 1/M_pp) to LDS, double-buffered so
// one barrier per pivot suffices; every thread then reads 4 column and 4 row
// values (128-bit loads) and updates its 16 entries with one FMA each; only
// the pivot row and column are fixed up.  Iterating p as 4 q + s with s
// unrolled keeps every register index static.  P is symmetric, so entry
// (r, c) is read from and written to P[r * ld + c] (coalesced along c).
__global__ __launch_bounds__(IT) void k_inv128(const SmallInvTask* __restrict__ tasks) {
  __shared__ __align__(16) double rowp[2][IB];
  __shared__ __align__(16) double colp[2][IB];
  __shared__ double ipv[2];
  const SmallInvTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, tr = tid >> 5, tc = tid & 31, w = tk.w;
  double v[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * tr + i, c = 4 * tc + j;
      v[i][j] = (r < w && c < w) ? G(tk.P)[(size_t)r * tk.ld + c] : (r == c ? 1.0 : 0.0);
    }
  int bad = -1;
  for (int q = 0; q < IB / 4; ++q) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int p = 4 * q + s, buf = s & 1;
      if (tr == q) {
        *(double2*)&rowp[buf][4 * tc] = double2{v[s][0], v[s][1]};
        *(double2*)&rowp[buf][4 * tc + 2] = double2{v[s][2], v[s][3]};
        if (tc == q) ipv[buf] = 1.0 / v[s][s];
      }
      if (tc == q) {
        *(double2*)&colp[buf][4 * tr] = double2{v[0][s], v[1][s]};
        *(double2*)&colp[buf][4 * tr + 2] = double2{v[2][s], v[3][s]};
      }
      __syncthreads();
      const double piv = rowp[buf][p];
      const double ip = ipv[buf];
      if (!(piv > 0.0) && bad < 0) bad = p;
      const double2 c01 = *(const double2*)&colp[buf][4 * tr];
      const double2 c23 = *(const double2*)&colp[buf][4 * tr + 2];
      const double2 r01 = *(const double2*)&rowp[buf][4 * tc];
      const double2 r23 = *(const double2*)&rowp[buf][4 * tc + 2];
      const double col[4] = {c01.x, c01.y, c23.x, c23.y};
      const double rc[4] = {r01.x * ip, r01.y * ip, r23.x * ip, r23.y * ip};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = fma(-col[i], rc[j], v[i][j]);
      if (tc == q) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i][s] = col[i] * ip;
      }
      if (tr == q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[s][j] = rc[j];
        if (tc == q) v[s][s] = -ip;
      }
    }
  }
  if (bad >= 0 && tid == 0) atomicCAS(tk.info, 0, tk.base + bad + 1);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * tr + i, c = 4 * tc + j;
      if (r < w && c < w) G(tk.P)[(size_t)r * tk.ld + c] = -v[i][j];
    }
}

void launch_inv128(const SmallInvTask* d_tasks, int n_tasks, hipStream_t s) {
  if (n_tasks > 0) k_inv128<<<n_tasks, IT, 0, s>>>(d_tasks);
}

// M (holding -A^-1 in its lower triangle) -> A^-1, full symmetric; 64 x 64
// tiles through LDS so both the lower and the mirrored upper writes coalesce.
// Grid (lower tiles of the largest block, tasks).
__global__ __launch_bounds__(256) void k_gj_finish(const InvTask* __restrict__ tasks) {
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
  for (int e = tid; e < 4096; e += 256) {  // lower tile (rows I, cols J), negated in place
    const int r = e % 64, c = e / 64;
    const size_t at = (size_t)(J * 64 + c) * np + I * 64 + r;
    if (I == J && r < c) continue;
    const double v = -G(tk.M)[at];
    G(tk.M)[at] = v;
    T[c * 65 + r] = v;
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {  // upper tile (rows J, cols I): (J+c, I+r) = (I+r, J+c)
    const int c = e % 64, r = e / 64;
    if (I == J && c >= r) continue;  // diagonal tile: only its strict upper part
    G(tk.M)[(size_t)(I * 64 + r) * np + J * 64 + c] = T[c * 65 + r];
  }
}

void launch_gj_finish(const InvTask* d_tasks, int n_tasks, int max_np, hipStream_t s) {
  const int nt = max_np / 64;
  if (n_tasks > 0 && nt > 0)
    k_gj_finish<<<dim3(nt * (nt + 1) / 2, n_tasks), 256, 0, s>>>(d_tasks);
}

// ---------------------------------------------------------------------------
// Outer (block 128) level of the sweep.  Tiles are 64 x 64.
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

// Bt[c, r] = M[r, kb + c] (from the lower triangle; Bt is w x np, ld w, the
// transposed column block), P[c, r'] = M[kb + r', kb + c] (w x w, ld w).
// Tiles: (np/64) x (w/64) over (row block r0 of M, column c0 of the block).
__global__ __launch_bounds__(256) void k_gj2_gather(const Gj2Task* __restrict__ tasks,
                                                    int n_tasks) {
  __shared__ double T[64 * 65];
  const Gj2Task tk = tasks[find_task(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int tw = tk.w / 64;
  const int r0 = (tile / tw) * 64, c0 = (tile % tw) * 64;
  const int np = tk.np, tid = threadIdx.x;
  const int col0 = tk.kb + c0;  // global column of the tile
  if (r0 >= col0 + 64) {
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      T[c * 65 + r] = G(tk.M)[(size_t)(col0 + c) * np + r0 + r];
    }
  } else if (r0 + 64 <= col0) {  // strictly above: read the transposed lower tile
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;
      T[c * 65 + r] = G(tk.M)[(size_t)(r0 + r) * np + col0 + c];
    }
  } else {  // diagonal tile
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      const int gr = r0 + r, gc = col0 + c;
      T[c * 65 + r] = gr >= gc ? G(tk.M)[(size_t)gc * np + gr] : G(tk.M)[(size_t)gr * np + gc];
    }
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {  // Bt column r0 + r holds row r0 + r of B
    const int c = e % 64, r = e / 64;
    G(tk.B)[(size_t)(r0 + r) * tk.w + c0 + c] = T[c * 65 + r];
  }
  if (r0 + 64 > tk.kb && r0 < tk.kb + tk.w) {  // the pivot rows: P is symmetric
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;
      G(tk.P)[(size_t)(r0 - tk.kb + r) * tk.w + c0 + c] = T[c * 65 + r];
    }
  }
}

// Swept row/column block from Ut = P^-1 Bt (w x np, ld w):
//   M[r, kb + c] = Ut[c, r] for r >= kb + w (below the pivot, lower storage),
//   M[kb + c, j] = Ut[c, j] for j < kb (stored at column j, row kb + c),
//   M[kb + r, kb + c] = -P^-1[r, c].
// Tiles: (np/64) x (w/64) over (row block r0, column c0 of the block).
__global__ __launch_bounds__(256) void k_gj2_fix(const Gj2Task* __restrict__ tasks, int n_tasks) {
  __shared__ double T[64 * 65];
  const Gj2Task tk = tasks[find_task(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int tw = tk.w / 64;
  const int r0 = (tile / tw) * 64, c0 = (tile % tw) * 64;
  const int np = tk.np, tid = threadIdx.x, kb = tk.kb, w = tk.w;
  if (r0 >= kb + w) {  // below the pivot: transpose through LDS so both sides coalesce
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;
      T[c * 65 + r] = G(tk.U)[(size_t)(r0 + r) * w + c0 + c];
    }
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      G(tk.M)[(size_t)(kb + c0 + c) * np + r0 + r] = T[c * 65 + r];
    }
  } else if (r0 < kb) {  // left of the pivot: row block kb.., columns r0..
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;
      G(tk.M)[(size_t)(r0 + r) * np + kb + c0 + c] = G(tk.U)[(size_t)(r0 + r) * w + c0 + c];
    }
  } else {  // pivot block
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      G(tk.M)[(size_t)(kb + c0 + c) * np + r0 + r] = -G(tk.P)[(size_t)(c0 + c) * w + (r0 - kb) + r];
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
// Restricted-stencil products: out = alpha Q_R (M + M2) + beta In (M2 optional,
// summed as M is loaded; + the sparse terms
// gamma Q_R + diag(dv) + I on the padded diagonal, added by k_sparse_add);
// rows are region nodes (padded to np).  Column c of the result is the
// 13-point stencil applied to column c of M, a field over the region.
//
// Workgroup = 256 output rows (one per thread) x up to 4 groups of 16
// columns.  The rows of M those outputs reach form one contiguous span
// [lo, hi] of region indices (the region is ordered by grid rows; a stencil
// reaches two grid rows up and down).  Per group, the span of its 16 columns
// is staged in LDS and the 13 taps are read from there; the loads of the next
// group are in flight (in registers) while the current one is computed.  The
// stencil rows (neighbours, coefficients) are loaded once per workgroup.  A
// tile whose span exceeds kRsSpan (a region more than 68 nodes wide) reads its
// taps from global memory.  tstore: write the result transposed
// (out[a * ldout + c], In read the same way; 16-byte stores when beta = 0).
// ---------------------------------------------------------------------------
namespace {
constexpr int kRsRows = 256, kRsCols = 16, kRsGroups = 4, kRsSpan = 528;
}

// kTwo: some task of the launch has a second input M2.  Its loads stay
// unconditional: a task without M2 reads M a second time with weight 0.
template <bool kTwo>
__global__ __launch_bounds__(256, 2) void k_rstencil(const StencilTask* __restrict__ tasks,
                                                  int n_tasks) {
  __shared__ double src[kRsCols * kRsSpan];
  __shared__ int span_lo, span_hi;
  int lo_t = 0, hi_t = n_tasks - 1;
  const int b = blockIdx.x;
  while (lo_t < hi_t) {
    int mid = (lo_t + hi_t + 1) / 2;
    if (tasks[mid].tile_start <= b) lo_t = mid; else hi_t = mid - 1;
  }
  const StencilTask tk = tasks[lo_t];
  const RegionDev rg = *tk.rg;
  const int tile = b - tk.tile_start;
  constexpr int kWide = kRsCols * kRsGroups;
  const int tiles_c = (tk.ncols + kWide - 1) / kWide;
  const int a0 = (tile / tiles_c) * kRsRows, cw = (tile % tiles_c) * kWide;
  const int ngrp = min(kRsGroups, (tk.ncols - cw + kRsCols - 1) / kRsCols);
  const int tid = threadIdx.x;
  const int a = a0 + tid;
  const bool use = tk.alpha != 0.0;
  const bool real = use && a < rg.nb;
  int nbr[kNS];
  double cf[kNS];
  int lo = INT_MAX, hi = -1;
  if (real) {
    const int node = G(rg.nodes)[a];
#pragma unroll
    for (int q = 0; q < kNS; ++q) {
      nbr[q] = G(rg.nbr)[a * kNS + q];
      cf[q] = G(tk.qs)[(size_t)q * tk.ns + node];
      if (nbr[q] >= 0) {
        lo = min(lo, nbr[q]);
        hi = max(hi, nbr[q]);
      }
    }
  }
  if (tid == 0) {
    span_lo = INT_MAX;
    span_hi = -1;
  }
  __syncthreads();
  if (real) {
    atomicMin(&span_lo, lo);
    atomicMax(&span_hi, hi);
  }
  __syncthreads();
  const int slo = span_lo, span = span_hi - span_lo + 1;  // span <= 0: no taps
  const bool staged = span > 0 && span <= kRsSpan;
  const bool row_ok = a < rg.np;
  const gptr<const double> m2 = G(tk.M2 ? tk.M2 : tk.M);
  const double w2 = tk.M2 ? 1.0 : 0.0;
  // entry (r, c) of the input M (+ M2)
  auto in_at = [&](size_t off) {
    return kTwo ? fma(w2, m2[off], G(tk.M)[off]) : G(tk.M)[off];
  };
  double ld[2 * kRsCols];
  double ld2[kTwo ? 2 * kRsCols : 1];
  // loads of group g: rows tid and tid + 256 of the span, 16 columns.  The
  // loads are unconditional (all in flight at once): a lane outside the span
  // or the columns reads entry (slo, c0), which exists; LDS entries outside
  // the span and the columns are never read by the taps.
  auto issue = [&](int g) {
    const int c0 = cw + g * kRsCols, ncc = min(kRsCols, tk.ncols - c0);
    const size_t safe = (size_t)c0 * tk.ldm + slo;
#pragma unroll
    for (int cc = 0; cc < kRsCols; ++cc) {
      const size_t mc = (size_t)(c0 + cc) * tk.ldm + slo;
      const size_t o0 = (cc < ncc && tid < span) ? mc + tid : safe;
      const size_t o1 = (cc < ncc && tid + 256 < span) ? mc + tid + 256 : safe;
      ld[2 * cc] = G(tk.M)[o0];
      ld[2 * cc + 1] = G(tk.M)[o1];
      if constexpr (kTwo) {
        ld2[2 * cc] = m2[o0];
        ld2[2 * cc + 1] = m2[o1];
      }
    }
  };
  if (staged) issue(0);
  for (int g = 0; g < ngrp; ++g) {
    const int c0 = cw + g * kRsCols, ncc = min(kRsCols, tk.ncols - c0);
    if (staged) {
      __syncthreads();  // the previous group is no longer read from src
#pragma unroll
      for (int cc = 0; cc < kRsCols; ++cc) {
        if constexpr (kTwo) {
          src[cc * kRsSpan + tid] = fma(w2, ld2[2 * cc], ld[2 * cc]);
          src[cc * kRsSpan + tid + 256] = fma(w2, ld2[2 * cc + 1], ld[2 * cc + 1]);
        } else {
          src[cc * kRsSpan + tid] = ld[2 * cc];
          src[cc * kRsSpan + tid + 256] = ld[2 * cc + 1];
        }
      }
      for (int e = tid; e < ncc * (span - 512); e += 256) {  // rows 512.. of a long span
        const int w = span - 512, cc = e / w, r = 512 + (e - cc * w);
        src[cc * kRsSpan + r] = in_at((size_t)(c0 + cc) * tk.ldm + slo + r);
      }
      __syncthreads();
      if (g + 1 < ngrp) issue(g + 1);
    }
    double v[kRsCols];
#pragma unroll
    for (int cc = 0; cc < kRsCols; ++cc) {
      double acc = 0.0;
      if (real && cc < ncc) {
        if (staged) {
#pragma unroll
          for (int q = 0; q < kNS; ++q)
            if (nbr[q] >= 0) acc += cf[q] * src[cc * kRsSpan + nbr[q] - slo];
        } else {
          const size_t mc = (size_t)(c0 + cc) * tk.ldm;
#pragma unroll
          for (int q = 0; q < kNS; ++q)
            if (nbr[q] >= 0) acc += cf[q] * in_at(mc + nbr[q]);
        }
        acc *= tk.alpha;
      }
      v[cc] = acc;
    }
    if (!row_ok) continue;
    if (!tk.tstore) {
#pragma unroll
      for (int cc = 0; cc < kRsCols; ++cc) {
        if (cc >= ncc) break;
        double r = v[cc];
        if (tk.beta != 0.0) r += tk.beta * G(tk.In)[(size_t)(c0 + cc) * tk.ldin + a];
        G(tk.out)[(size_t)(c0 + cc) * tk.ldout + a] = r;
      }
    } else if (ncc == kRsCols && tk.beta == 0.0) {  // 16 contiguous doubles of row a
      const gptr<double> o = G(tk.out) + (size_t)a * tk.ldout + c0;
#pragma unroll
      for (int k = 0; k < kRsCols / 2; ++k) stg2(o + 2 * k, v[2 * k], v[2 * k + 1]);
    } else {
#pragma unroll
      for (int cc = 0; cc < kRsCols; ++cc) {
        if (cc >= ncc) break;
        double r = v[cc];
        if (tk.beta != 0.0) r += tk.beta * G(tk.In)[(size_t)a * tk.ldin + c0 + cc];
        G(tk.out)[(size_t)a * tk.ldout + c0 + cc] = r;
      }
    }
  }
}

int rstencil_tiles(int np, int ncols) {
  return ((np + kRsRows - 1) / kRsRows) * ((ncols + kRsCols * kRsGroups - 1) / (kRsCols * kRsGroups));
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
    const int node = G(rg.nodes)[a];
    if (tk.gamma != 0.0)
      for (int q = 0; q < kNS; ++q) {
        const int c = G(rg.nbr)[a * kNS + q];
        if (c >= 0) G(tk.out)[(size_t)c * tk.ldout + a] += tk.gamma * qs[(size_t)q * ns + node];
      }
    if (tk.dv) G(tk.out)[(size_t)a * tk.ldout + a] += G(tk.dv)[node];
  } else if (tk.pad_identity) {
    G(tk.out)[(size_t)a * tk.ldout + a] += 1.0;
  }
}

void launch_rstencil(const StencilTask* d_tasks, int n_tasks, int total_tiles, int max_np,
                     int two, hipStream_t s) {
  if (total_tiles <= 0) return;
  if (two)
    k_rstencil<true><<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
  else
    k_rstencil<false><<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
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
    T[c * 65 + r] = G(tk.M)[(size_t)(J * 64 + c) * np + I * 64 + r];
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {  // upper tile (rows J, cols I): M[J+c, I+r] = T[c][r]
    const int c = e % 64, r = e / 64;
    if (I == J && c >= r) continue;  // diagonal tile: only its strict upper part
    G(tk.M)[(size_t)(I * 64 + r) * np + J * 64 + c] = T[c * 65 + r];
  }
}

void launch_mirror(const InvTask* d_tasks, int n_tasks, int max_np, hipStream_t s) {
  const int nt = max_np / 64;
  if (n_tasks > 0 && nt > 0) k_mirror<<<dim3(nt * (nt + 1) / 2, n_tasks), 256, 0, s>>>(d_tasks);
}

}  // namespace rbmc
