// Internal declarations of the RBMC library (host runtime + HIP kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rbmc.h"

namespace rbmc {

// 13-point spatial stencil of Q_s (|dx| + |dy| <= 2), fixed order.
constexpr int kNS = 13;
constexpr int kSdx[kNS] = {0, -1, 1, 0, 0, -2, 2, 0, 0, -1, 1, -1, 1};
constexpr int kSdy[kNS] = {0, 0, 0, -1, 1, 0, 0, -2, 2, -1, -1, 1, 1};
// the first 5 entries form the 5-point stencil of G, K_kappa and F_s
constexpr int kN5 = 5;

// Global-memory views of device pointers.  Pointers read from task records
// are generic, so accesses through them compile to flat instructions, which
// count against the LDS wait counter as well: a wait for LDS reads would then
// also wait for a global prefetch in flight.  Accesses through these views
// compile to global instructions.  Only for pointers into device memory.
template <class T>
using gptr = T __attribute__((address_space(1)))*;
template <class T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}
typedef double gv2d __attribute__((ext_vector_type(2)));
// 16-byte global load / store of two consecutive doubles
__device__ __forceinline__ double2 ldg2(gptr<const double> p) {
  const gv2d v = *(gptr<const gv2d>)p;
  return double2{v.x, v.y};
}
__device__ __forceinline__ void stg2(gptr<double> p, double x, double y) {
  *(gptr<gv2d>)p = gv2d{x, y};
}

// Dense blocks are padded to multiples of this (identity on the padded diagonal).
constexpr int kPad = 64;
inline int pad_to(int n) { return (n + kPad - 1) / kPad * kPad; }

// ---------------------------------------------------------------------------
// Planner (host, integer)
// ---------------------------------------------------------------------------

struct Region {  // spatial node set R with its restricted 13-point stencil
  int x0, x1, y0, y1, hops;      // core box and L1 growth 2*hops
  std::vector<int> nodes;        // global spatial ids, ascending
  std::vector<int> nbr;          // nodes.size() x kNS local ids, -1 = not in R
  std::vector<uint8_t> in_box;   // node lies in the core box
  int nb() const { return (int)nodes.size(); }
};

struct Chain {  // block-tridiagonal principal submatrix: time range x region
  int region;
  int t0, T;            // global time range [t0, t0+T)
  int ct0, cT;          // core time range (global) within the chain
  int core_id;          // core p (or -1)
};

struct Plan {
  int mx, my, T, ns, n;
  int P, ntx, nty, hops;
  int sep = 0;                // Alg. 2: separator layers between the cores
  std::vector<int> sep_nodes;  // their global node ids, ascending (sep = 1)
  std::vector<int> slab_t0, slab_len, tile_x0, tile_xlen, tile_y0, tile_ylen;
  std::vector<Region> regions;
  std::vector<Chain> sub;  // RBMC subdomains Omega_p* (one per core)
  std::vector<Chain> bj;   // block-Jacobi cores Omega_p
};

int piece_start(int idx_piece, int len, int parts);
int piece_len(int idx_piece, int len, int parts);
std::string make_plan(const rbmc_model_desc& d, const rbmc_decomp_desc& dc, Plan& plan);
void plan_labels(const Plan& plan, int32_t* label);
void plan_state(const Plan& plan, int p, uint8_t* state);

// ---------------------------------------------------------------------------
// Model coefficients
// ---------------------------------------------------------------------------

struct Coefs {
  double kappa, tau, rho, sigma, h;
  std::vector<double> qs;    // kNS x ns  Q_s
  std::vector<double> kk;    // kN5 x ns  dQ_s/dlog kappa = tau (4 kappa^4 C + 4 kappa^2 G)
  std::vector<double> fs;    // kN5 x ns  F_s = sqrt(tau) (kappa^2 C + G) C^-1/2
  std::vector<double> qd, dqd, ld;  // per time step: Q_t diagonal, dQ_t/drho diagonal, L_tt
  double qo, dqo, lo;        // Q_t off-diagonal, its rho-derivative, L_{t+1,t}
  double dobs;               // sigma^-2
};
void make_coefs(int mx, int my, int T, double h, double log_kappa, double log_tau, double rho,
                double log_sigma, Coefs& c);

// ---------------------------------------------------------------------------
// Kernel launch interfaces (kernels_*.hip)
// ---------------------------------------------------------------------------

struct DevModel {  // device views used by the stencil kernels
  int mx, my, T, ns, n, n_obs;
  const double* qs;   // kNS x ns
  const double* kk;   // kN5 x ns
  const double* fs;   // kN5 x ns
  const double* qd;   // T
  const double* dqd;  // T
  const double* ld;   // T
  double qo, dqo, lo;
  const double* dvec;     // n: sigma^-2 * mask
  const int* obs_rank;    // n: rank among observed (or -1)
  // the mask as bits (n / 32 words; small enough to stay in L2 across the
  // columns of a launch), the observed nodes before each word, sigma^-2
  const uint32_t* obs_bits;
  const int* obs_wrank;
  double dobs;
  // spectral preconditioner (set when the model has it): orthonormal DCT-II
  // matrices (column-major, C[k, i] = c_k cos(pi k (2 i + 1) / (2 m))), the
  // per-frequency time recursion (c'_t, 1 / den_t at t ns + f; the
  // off-diagonal lambda_f q_o at f) and whether the 2-D transforms run as
  // matrix-core GEMMs (sizes multiples of 16, at least 64) or by the direct kernel
  const double* dct_x;    // mx x mx
  const double* dct_y;    // my x my
  const double* sp_cp;    // T x ns
  const double* sp_id;    // T x ns
  const double* sp_off;   // ns
  int spec_gemm;  // transformed outside the direct DCT kernel (FFT or GEMM route)
};

// node i observed; its rank among the observed nodes (valid when observed)
__device__ __forceinline__ bool obs_at(const DevModel& m, size_t i) {
  return (m.obs_bits[i >> 5] >> (i & 31)) & 1u;
}
__device__ __forceinline__ int obs_rank_at(const DevModel& m, size_t i) {
  return m.obs_wrank[i >> 5] + __popc(m.obs_bits[i >> 5] & ((1u << (i & 31)) - 1u));
}

// Column sets: the sampler works on the columns (model, sample) of one or
// many models at once.  Column c has length len[c] (the model's n), starts at
// off[c] in the concatenated multi-vectors, reads its operator input at
// in_off[c] (for F the input column has n + n_obs entries) and belongs to
// model[c] (index into the device array of DevModel).
struct ColSet {
  int ncols;
  int max_len;
  int max_tiles;             // stencil tiles of the largest model
  int max_ns;                // spatial nodes of the largest model
  int max_T;                 // time steps of the longest model
  const int64_t* off;
  const int64_t* in_off;
  const int* len;
  const int* model;
  const DevModel* dms;
};

// One axis of the orthonormal DCT-II (inverse = 0) or DCT-III (inverse = 1)
// of nslices 2-D slices by FFT: nl lines of length N = 2^lg per slice, line
// l of slice q at q sstride + l lstride, elements estride apart.  tw: N/2
// pairs (cos, sin)(2 pi t / N); ph: N pairs (cos, sin)(pi k / 2N).
struct FftTask {
  const double* in;
  double* out;
  const double* tw;
  const double* ph;
  int N, lg, nl, nslices;
  long sstride, lstride, estride;
  int inverse;
  int tile_start;
};
bool fft_length_ok(int N);
int fft_tiles(int N, long lines);
void launch_dct_fft(const FftTask* d_tasks, int n_tasks, int total_tiles, int axis, int max_n,
                    hipStream_t s);

int stencil_tiles(int mx, int my);
// load the operator kernels' code object now (an empty launch on s)
void load_stencil_module(hipStream_t s);
// y = Op x per column (op = RBMC_OP_*), x at in_off, y at off
void launch_apply_op(const ColSet& cs, int op, const double* x, double* y, hipStream_t s);
// q = Q p per column and partial sums of p.q: partial[c * max_tiles + tile]
void launch_spmm_dot(const ColSet& cs, const double* p, double* q, double* partial,
                     hipStream_t s);

// PCG helpers (per-column scalars on the device)
void launch_reduce_partials(const double* partial, int nchunk, int n_rhs, double* out,
                            hipStream_t s);
int dot_chunks(int n);
void launch_dot_partials(const ColSet& cs, const double* a, const double* b, double* partial,
                         hipStream_t s);
void launch_pcg_xr(const ColSet& cs, const double* p, const double* q, double* x, double* r,
                   const double* rz, const double* pq, const uint8_t* active,
                   double* rr_partial, hipStream_t s);
// beta = (rz_new - rz_sub) / rz_old when rz_sub is given (flexible PCG)
void launch_pcg_p(const ColSet& cs, const double* z, double* p, const double* rz_new,
                  double* rz_old, const uint8_t* active, int first, hipStream_t s,
                  const double* rz_sub = nullptr);
void launch_pcg_check(const double* rr, const double* bb, double rtol, uint8_t* active,
                      int* it_count, int* n_active, int n_rhs, hipStream_t s);

// Chain-panel kernels (dense blocks padded to np = pad_to(nb), identity pad)
struct RegionDev {
  int nb, np;
  const int* nodes;      // nb
  const int* nbr;        // nb x kNS
  const uint8_t* in_box; // nb: node lies in the core box
};

// grouped GEMM: C = alpha * op(A) * op(B) + beta * Cin  (FP64 MFMA)
struct GemmTask {
  const double* A;
  const double* B;
  const double* Cin;
  double* C;
  int M, N, K;
  int lda, ldb, ldc, ldcin;
  double alpha, beta;
  int transA, transB;
  int tiles_n;
  int tile_start;
  int lower;          // 1: square C, only 128-tiles with row index >= column index
  int skip0, skip1;   // tiles meeting rows or columns [skip0, skip1) are skipped
};
// tiles of ts x ts (lower: only tiles with row index >= column index)
int gemm_task_tiles(int M, int N, int lower, int ts);
// kernels: FP64 128 x 128 tiles; FP64 64 x 64 tiles (for launches with few
// tiles); FP32 matrix-core products with FP64 accumulation across K chunks
// (128 x 128 tiles)
enum { kGemmF64 = 0, kGemmSmall = 1, kGemmMixed = 2 };
// tag 1: the spectral transforms (a separately named instantiation of the
// same FP64 kernel)
void launch_gemm(const GemmTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s,
                 int kind, int tag = 0);

// Gauss-Jordan sweep inversion of SPD matrices (in place).
struct InvTask {
  double* M;     // np x np col-major, ld = np
  int np;
  int nb;        // unpadded size (for work accounting)
  int* info;
};
// M (holding -A^-1 in its lower triangle) -> A^-1, full symmetric
void launch_gj_finish(const InvTask* d_tasks, int n_tasks, int max_np, hipStream_t s);

// Register-resident sweep of a block of order w <= 128 (full symmetric,
// column-major, leading dimension ld): P <- P^-1.  A non-positive pivot p
// sets *info = base + p + 1 (if still 0).
struct SmallInvTask {
  double* P;
  int w, ld;
  int* info;
  int base;
};
void launch_inv128(const SmallInvTask* d_tasks, int n_tasks, hipStream_t s);

// Outer level (block w = 128 or 256) of the sweep for large blocks: gather
// the column block [kb, kb + w) of M (lower-stored) transposed into B (w x np,
// ld w) and the pivot block into P (w x w, ld w); after P <- P^-1 and
// U = P B (w x np: the transposed panel P^-1 B^T), the GEMM updates the lower
// tiles (M -= U^T B) and the fix pass writes the swept row/column block.
// Both panels are kept transposed so every product reads its operands in
// the GEMM's fast orientation.
struct Gj2Task {
  double* M;
  double* B;   // w x np
  double* U;   // w x np
  double* P;   // w x w
  int np, kb, w;
  int tile_start;
};
void launch_gj2_gather(const Gj2Task* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
void launch_gj2_fix(const Gj2Task* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
int gj2_tiles(int np, int w);

// restricted-stencil products on dense column-major matrices (rows = region nodes):
//   out = alpha * Q_R * op(M) + gamma * Q_R + diag(dv) (+ I on pad) + beta * In
struct StencilTask {
  const double* M;     // np x ncols, column-major (ldm); may be null (alpha = 0)
  const double* M2;    // optional second input of the same shape: Q_R (M + M2)
  const double* In;    // optional (beta)
  double* out;
  int ldm, ldin, ldout;
  int ncols;           // number of columns of the result (np for square, n_k for panels)
  int tstore;          // store the result transposed: out[a * ldout + c] (In read the same way)
  double alpha, beta, gamma;
  const double* dv;    // optional diagonal (indexed by spatial node), square only
  int pad_identity;    // add 1 on padded diagonal (square only)
  const RegionDev* rg; // device pointer
  const double* qs;    // the model's Q_s stencil (kNS x ns)
  int ns;
  int tile_start;
};
// output tiles of one task (np rows x ncols)
int rstencil_tiles(int np, int ncols);
// max_np > 0: also add the sparse terms (gamma Q_R, diag(dv), pad identity);
// two: some task has a second input M2
void launch_rstencil(const StencilTask* d_tasks, int n_tasks, int total_tiles, int max_np,
                     int two, hipStream_t s);
// copy the lower triangle of each task's M (np x np) onto its upper triangle
void launch_mirror(const InvTask* d_tasks, int n_tasks, int max_np, hipStream_t s);

// Panel transfers between global multi-vectors (column k of the model at
// X + k n) and chain panels (np x n_k, ld np): mode 0 gather (pad rows
// zeroed), 1 scatter, 2 correction right-hand side r = Q_AB x_B for the block
// at global time t of a chain whose time range is [t0, t0 + T).
struct PanelTask {
  double* P;
  const RegionDev* rg;
  const DevModel* dm;
  const double* X;   // source multi-vector (modes 0, 2)
  double* Xout;      // destination multi-vector (mode 1)
  int n_k;
  int t;        // global time step of the block
  int t0, T;    // chain time range (modes 2, 3)
  // mode 0: P = X at step t (gather); 1: Xout = P (scatter); 2: P = Q_AB x_B
  // at step t of the chain [t0, t0 + T) x R; 3: its part from spatial
  // neighbours outside R (any step); 4: P += w X at step t (gather, add)
  int mode;
  // modes 2, 3: rows (nullptr: all np rows of R, panel leading dimension np)
  // or a list of ld region rows (-1: a zero row), the panel then ld x n_k
  const int* rows;
  int ld;
  double w;     // mode 4
  int tile_start;
};
void launch_panels(const PanelTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
int panel_tiles(int np, int n_k);

// Deterministic part of the outputs from dense blocks of Q_AA^-1:
//   kind 0 (diagonal block Sigma_tt): diag_out[t*ns + node] = Sigma_aa on core
//     nodes; sums D_a Sigma_aa, <Sigma, Q_s>_F, <Sigma, K>_F over core rows;
//   kind 1 (off-diagonal block given as X with Sigma_off = sign * op(X)):
//     the two Frobenius products.
// Partial sums of chunk c go to partial[(out_index + c) * 3 + j].
struct ExtractTask {
  const double* M;
  int ld;
  const RegionDev* rg;
  const DevModel* dm;
  double* diag_out;
  double* partial;
  int out_index;
  int t;          // global time of the rows
  int kind;
  int trans;
  double sign;
  int tile_start;
};
void launch_extract(const ExtractTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
// Off-diagonal time-block entries on the stencil pattern of the core rows:
// Sigma_{t,t'}[a, c] = scale * W[:, c] . Sigma_tt[:, a] (both column-major,
// ld), accumulated like k_extract's off-diagonal slots (partial chunk layout
// identical).  One tile = 256 region rows.
struct OffdiagTask {
  const double* W;
  const double* Sig;
  int ld;
  const RegionDev* rg;
  const DevModel* dm;
  double* partial;
  int out_index;
  double scale;
  int tile_start;
};
void launch_offdiag(const OffdiagTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);

// Monte Carlo part from the correction panels mu_t (np x n_k) of a chain, with
// scale = 1 / (the estimate's total number of samples; n_k when it is drawn
// in one pass):
//   diag_out[t*ns + node] += scale sum_k mu_t[a,k]^2 on core nodes;
//   partial sums of scale sum_k mu_t[a,k] (S mu_t')[a,k] for t' = t-1, t, t+1,
//   S in {Q_s, K}, of scale sum_k D_a mu_t[a,k]^2 and of m_a / s2_a (the last
//   meaningful only for a one-pass estimate).
// Partial sums of chunk c (region rows [256 c, 256 c + 256)) go to
// partial[(out_index + c) * 8 + j] (added to the previous value when accum
// is set); a task spans mc_chunks(np) chunks.
__host__ __device__ inline int mc_chunks(int np) { return (np + 255) / 256; }
// With stack set, the task covers `steps` (<= 4) consecutive core steps from
// local step tl: panel u of the chain (u < ta) at stack + u np n_k, partial
// sums of step s at out_index + s mc_chunks(np), diagonal at step t + s.
struct McTask {
  const double* mu[3];  // panels for t-1, t, t+1 (null if outside the chain)
  const double* stack;  // or the chain's stacked panels
  int ta, tl, steps;
  double scale;         // 1 / (total samples of the estimate)
  int accum;            // add to the partial sums (later sample passes)
  int np;
  const RegionDev* rg;
  const DevModel* dm;
  double* diag_out;
  double* partial;
  int out_index;
  int n_k;
  int t;
  int tile_start;
};
// multi: tasks of several steps (their windows of (steps + 2) panels x the
// region's widest 256-row span fit in mc_lds_doubles() for one sample)
void launch_mc(const McTask* d_tasks, int n_tasks, int total_tiles, int multi, hipStream_t s);
int mc_max_steps();
// Alg. 2 separator variance (see k_sep_var)
void launch_sep_var(const int* sep, int nsep, const double* x, long ldx, int nk, double scale,
                    int accum, double* diag, hipStream_t s);
int mc_lds_doubles();

// ---------------------------------------------------------------------------
// Learned correction to the preconditioner: 3-D convolutions (kernels_conv.hip)
// ---------------------------------------------------------------------------
struct ConvGeom {  // volume of T x MY x MX voxels
  int T, MY, MX;
};
struct ConvBox {  // valid voxels [t0, t1) x [y0, y1) x [x0, x1) of one volume
  int t0, t1, y0, y1, x0, x1;
};
struct ConvArgs {
  const float* in;        // B x Cin x V
  float* out;             // B x Cout x V
  const uint16_t* w;      // Cout x Cin x 27, BF16
  const float* mask;      // optional, B x Cout x V: outputs where mask <= 0 are zeroed
  const ConvBox* boxes;   // optional (device), one per volume; null = whole volume
  ConvGeom geom;
  int relu_in;            // apply max(0, .) to the input on load
  int accumulate;         // out += result
  float scale;
};
int conv_tiles(const ConvGeom& g);
void launch_conv3d(const ConvArgs& a, int cin, int cout, int batch, hipStream_t s);
struct ConvWArgs {
  const float* gout;      // B x Cout x V
  const float* ain;       // B x Cin x V
  float* partial;         // (tiles * B) x Cout x Cin x 27
  const ConvBox* boxes;
  ConvGeom geom;
  int relu_in;
};
int conv_wgrad_tiles(const ConvGeom& g);
void launch_conv3d_wgrad(const ConvWArgs& a, int cin, int cout, int batch, hipStream_t s);
void launch_sum_rows(const float* part, int nwg, int len, float* out, hipStream_t s);
void launch_conv_wflip(const uint16_t* w, int cin, int cout, uint16_t* wt, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int n, float lr,
                 float b1, float b2, float eps, int step, hipStream_t s);
void launch_to_bf16(const float* p, uint16_t* pb, int n, hipStream_t s);
// two-channel network input (r, u) / sqrt(rr[c]) from FP64 columns; output back
void launch_cols2_to_vol(const double* r, const double* u, size_t n, const double* rr, float* vol,
                         int ncols, hipStream_t s);
void launch_vol_to_cols(const float* vol, size_t n, const double* rr, const uint8_t* active,
                        double* y, int ncols, int accumulate, hipStream_t s);
// training pairs, batches and the energy loss
void launch_pair_store(const double* r, const double* u, const double* xs, const double* x,
                       size_t n, const double* rr, const int* slot, float* R, float* U, float* E,
                       int ncols, hipStream_t s);
void launch_pack_train(const float* R, const float* U, const int* slots, size_t n, float su,
                       float* vin, int batch, hipStream_t s);
void launch_energy_d(const float* U, const float* E, const float* y, const int* slots, size_t n,
                     float inv_su, double* d, int batch, hipStream_t s);
void launch_energy_dot(const double* a, const float* af, const int* slots, const double* q,
                       const float* qf, size_t n, const float* coef, float* gy, double* part,
                       int nblk, int batch, hipStream_t s);
// safeguarded correction z_c += g_c v_c, g_c = (vr - vqu) / vqv
void launch_gamma_axpy(const double* v, double* z, size_t n, const double* vr, const double* vqu,
                       const double* vqv, const uint8_t* active, int ncols, hipStream_t s);

// ---------------------------------------------------------------------------
// Spectral preconditioner M = Q_t (x) Q_s + dbar I (kernels_stencil.hip):
// per-frequency coefficients of the time recursion, the tridiagonal solves,
// and the direct 2-D DCT kernel for grids the GEMM route does not take.
// ---------------------------------------------------------------------------
struct SpecCoefTask {
  const double* lam;   // ns eigenvalues of Q_s (DCT order f = ky mx + kx)
  const double* qd;    // T
  double qo, dbar;
  int ns, T;
  double *cp, *id, *off;
};
void launch_spec_coef(const SpecCoefTask& t, hipStream_t s);
// in place on every column of the set (columns of spectral models only)
void launch_spec_solve(const ColSet& cs, double* y, hipStream_t s);
// y = transform of x along one axis (0: x, 1: y); inverse = 1 applies C^T;
// columns of models with spec_gemm set are skipped
void launch_dct_direct(const ColSet& cs, const double* x, double* y, int axis, int inverse,
                       hipStream_t s);

// ---------------------------------------------------------------------------
// Kronecker form of the subdomain inverse (kernels_kron.hip)
// ---------------------------------------------------------------------------
struct KronRegionTask {  // per region: dR, qR, kR from S^-1 (np x np)
  const double* inv;
  const RegionDev* rg;
  const DevModel* dm;
  double *dR, *qR, *kR;
  int tile_start;
};
void launch_kron_region(const KronRegionTask* d_tasks, int n_tasks, int total_tiles,
                        hipStream_t s);
// mode 0: Z = S^-1[:, a_o] (np x nc), zero columns where a_o = -1;
// mode 1: C (nc x nc) from Z
struct KronBuildTask {
  int mode;
  const double* inv;
  const double* Z;
  const double* V;     // TA x TA
  const int* obs_a;    // nc: region-local node of slot o, -1 unused
  const int* obs_t;    // nc: local time step of slot o
  double* out;
  int np, nc, TA;
  double noise;        // sigma^2 = D_o^-1
  int tile_start;
};
int kron_cols_tiles(int rows, int cols);
void launch_kron_build(const KronBuildTask* d_tasks, int n_tasks, int total_tiles,
                       hipStream_t s);
struct KronReduceTask {  // group sums of X_g against Z, KZ, the observed entries
  const double* X;
  const double* Z;
  const double* KZ;
  const int* obs_a;
  const int* goff;     // TA: first slot of each time group
  const int* gpad;     // TA: slots of each time group (multiple of 16)
  double* part;        // TA x TA x 3 x np
  int np, TA, g;
  int tile_start;
};
void launch_kron_reduce(const KronReduceTask* d_tasks, int n_tasks, int total_tiles,
                        hipStream_t s);
struct KronDetTask {  // deterministic entries at one core step t of a subdomain
  const double* V;
  const double* part;
  const double *dR, *qR, *kR;
  const RegionDev* rg;
  const DevModel* dm;
  double* diag_out;
  double* partial;
  int out_index, nchk;
  int TA, t, t0;
  int tile_start;
};
void launch_kron_det(const KronDetTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
struct KronMixTask {  // out_t = beta In_t + alpha sum_t' V[t,t'] U_t' over stacked panels
  const double* V;
  const double* U;
  const double* In;
  double* out;
  int np, n_k, TA;
  double alpha, beta;
  int tile_start;
};
int kron_mix_tiles(int np, int n_k);
void launch_kron_tmix(const KronMixTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
struct KronObsTask {  // v = observed entries of stacked panels U (nc x n_k)
  const double* U;
  double* v;
  const int* obs_a;
  const int* obs_t;
  int np, nc, n_k;
  int tile_start;
};
void launch_kron_obs(const KronObsTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s);
void launch_fill(double* p, size_t n, double value, hipStream_t s);
// element offset + i (i < count) of the standard-normal stream of seed
void launch_normals(uint64_t seed, uint64_t offset, size_t count, double* out, hipStream_t s);
// per-block sums of (diag - det) / diag over n nodes (mc_share_blocks(n) blocks)
int mc_share_blocks(size_t n);
void launch_mc_share(const double* diag, const double* det, size_t n, double* partial,
                     hipStream_t s);

// posterior mean with fixed effects (kernels_mean.hip)
constexpr int kMaxFixedEffects = RBMC_MAX_FIXED_EFFECTS;
// b (n x (nb + 1), column c at c ldb) = [A_u^T Q_y y, A_u^T Q_y A_beta]
void launch_mean_rhs(int n, int n_obs, const int* rank, double tau_y, const double* y,
                     const double* a, int nb, double* b, size_t ldb, hipStream_t s);
// out[j ny + c] = sum_{r < L} x_j[r] y_c[r] (column 0 of y at y0, column
// c >= 1 at y1 + (c - 1) ldy); part holds mean_gram_blocks(L) nx ny doubles
int mean_gram_blocks(int L);
void launch_mean_gram(int L, int nx, const double* x, size_t ldx, int ny, const double* y0,
                      const double* y1, size_t ldy, double* part, double* out, hipStream_t s);
// out: [status, mu_beta (nb), S^-1 (nb x nb)] from g = Q_betau [w, W],
// h = A_beta^T [y, A_beta] and the prior precisions q (1 <= nb <= 32)
void launch_mean_schur(int nb, const double* g, const double* h, const double* q, double tau_y,
                       double* out, hipStream_t s);
// mu_u = w - W mu_beta and var_add = diag(W S^-1 W^T) (var_add may be NULL)
void launch_mean_combine(int n, int nb, const double* w, size_t ldw, const double* sol,
                         double* mu_u, double* var_add, hipStream_t s);

}  // namespace rbmc
