// C ABI of the RBMC library and the host-side runtime that sequences the
// kernels: block-tridiagonal factorization of every chain (block-Jacobi blocks
// and RBMC subdomains), the selected inverse entries, the correction solves and the
// preconditioned conjugate-gradient sampler.
//
// Everything runs on *sets* of models: one model for the single-model calls,
// many uneven models for rbmc_estimate_batched.  Every launch covers all
// chains (and all sample columns) of the set, so a step of a recursion is one
// launch per kernel, not one per subdomain or per model.
#include <algorithm>
#include <array>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <fstream>
#include <mutex>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "rbmc_impl.h"

using namespace rbmc;

static thread_local std::string g_err;

static rbmc_status fail(rbmc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? RBMC_E_OOM : RBMC_E_DEVICE,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

namespace {

// Device allocations with a byte count.
struct Pool {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  hipError_t alloc(void** p, size_t n) {
    hipError_t e = hipMalloc(p, n ? n : 8);
    if (e == hipSuccess) {
      ptrs.push_back(*p);
      bytes += (int64_t)n;
    }
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

// Host-built task lists uploaded once per call; launches reference offsets.
struct Arena {
  std::vector<uint8_t> host;
  void* dev = nullptr;
  size_t cap = 0;
  template <class T>
  size_t push(const std::vector<T>& v) {
    size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  template <class T>
  T* at(size_t off) const {
    return (T*)((uint8_t*)dev + off);
  }
  hipError_t upload(hipStream_t s) {
    if (host.size() > cap) {
      if (dev) (void)hipFree(dev);
      dev = nullptr;
      cap = std::max(host.size() * 5 / 4, (size_t)1 << 20);
      hipError_t e = hipMalloc(&dev, cap);
      if (e != hipSuccess) {
        cap = 0;
        return e;
      }
    }
    if (host.empty()) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  void clear() { host.clear(); }
  ~Arena() {
    if (dev) (void)hipFree(dev);
  }
};

struct ProfRec {
  int family;
  hipEvent_t a, b;
  double flops, bytes;
};

}  // namespace

// Outer Gauss-Jordan step widths: rank-512 steps for batches of large blocks
// (longer products, half the re-reads of the updated matrix; measured faster
// than 256 on order-4096 blocks), 256 for batches of smaller blocks, 128 for
// one to three blocks (a shorter chain of dependent launches).  A chain's
// sweep workspaces are sized for the widest step its blocks take.
constexpr int kSweepMax = 512;
constexpr int kSweepWideFrom = 2048;  // smallest block order with rank-512 workspaces
inline int sweep_width_of(int np) {
  return np >= kSweepWideFrom ? kSweepMax : std::min(256, np);
}

// Launch-shape choices that the autotuner sets per context (rbmc_autotune):
// products with K <= small_k or fewer than small_tiles 128-tiles use the
// 64 x 64-tile GEMM; batches whose blocks all have order >= wide_from take
// rank-512 sweep steps (wide_from >= kSweepWideFrom, the workspace bound).
struct Tune {
  int small_k = 256;
  int small_tiles = 768;
  int wide_from = kSweepWideFrom;
};
// the tuning in force while programs are built on this thread
thread_local Tune g_tune;

struct rbmc_ctx {
  int device;
  hipStream_t stream;         // the caller's stream: all results are ordered on it
  // library streams of the overlapped estimate: the sampler and the
  // corrections (work), the subdomain factorization (side) and the core
  // steps (side2); the two side streams can be kept off `reserve_cus`
  // compute units so the sampler's chain of dependent launches always finds
  // free ones
  hipStream_t work = nullptr, side = nullptr, side2 = nullptr;
  int reserve_cus = 0;
  bool cu_masked = false;  // the side streams were created with a CU mask
  Tune tune;               // launch-shape choices (rbmc_autotune / rbmc_ctx_set_tune)
  hipEvent_t join[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  Arena arenaA, arenaB;       // task lists of work on the caller's / side stream
  // concatenated sample-column workspace of the sampler (sized per call)
  Pool ws;
  size_t ws_len = 0, ws_zlen = 0;
  int ws_cols = 0, ws_models = 0;
  double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *x = nullptr, *zcat = nullptr;
  double* zp = nullptr;        // previous preconditioned residual (flexible PCG)
  double* scal = nullptr;      // 9 x columns
  // learned correction v = N_w(r, u) and Q v per column (allocated on first use)
  Pool lws;
  size_t lws_len = 0;
  double *lv = nullptr, *lqv = nullptr;
  double* part = nullptr;      // column partial sums
  size_t part_len = 0;
  uint8_t* active = nullptr;
  int* iters = nullptr;        // columns + 1
  int64_t *d_off = nullptr, *d_in_off = nullptr;
  int *d_len = nullptr, *d_model = nullptr;
  DevModel* d_dms = nullptr;
  double* epart = nullptr;     // estimator partial sums
  size_t epart_len = 0;
  Pool epool;
  // workspace of the Kronecker method (a batch of subdomains at a time)
  Pool kws;
  char* kws_base = nullptr;
  size_t kws_cap = 0;
  size_t kron_batch_cap = 0;  // upper bound of a batch's workspace (0: free memory)
  Pool kbank;  // Y of every subdomain and the deterministic diagonals, kept across sample passes
  char* kbank_base = nullptr;
  size_t kbank_cap = 0;
  // scheduling of rbmc_estimate*: overlap the sampler with the subdomain
  // factorization + core steps on further streams (else one after the
  // other on the context stream), and enqueue the two streams from two host
  // threads (else from one)
  bool overlap = true;
  bool launch_threads = true;
  // instrumentation (records may be added from two host threads)
  bool prof = false;
  std::mutex prof_mu;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;

  hipEvent_t ev() {  // prof_mu held
    hipEvent_t e = nullptr;
    if (!spare.empty()) {
      e = spare.back();
      spare.pop_back();
    } else {
      (void)hipEventCreate(&e);
    }
    return e;
  }
  // bracket a launch sequence of one kernel family on stream s
  int begin(int family, double flops, double bytes, hipStream_t s) {
    if (!prof) return -1;
    std::lock_guard<std::mutex> lk(prof_mu);
    ProfRec r{family, ev(), ev(), flops, bytes};
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id, hipStream_t s) {
    if (id < 0) return;
    std::lock_guard<std::mutex> lk(prof_mu);
    (void)hipEventRecord(recs[id].b, s);
  }
  void clear() {
    for (ProfRec& r : recs) {
      spare.push_back(r.a);
      spare.push_back(r.b);
    }
    recs.clear();
  }
  ~rbmc_ctx() {
    clear();
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
    if (side2) (void)hipStreamDestroy(side2);
    if (work) (void)hipStreamDestroy(work);
    ws.release();
    epool.release();
    kws.release();
    kbank.release();
    kbank_base = nullptr;
    kbank_cap = 0;
  }
};

namespace {

// A set of block-tridiagonal chains with their dense blocks and workspaces.
// For one model the owner of every chain is that model; a batched call
// concatenates the sets of many models.

struct ChainSet {
  std::vector<Chain> chains;
  std::vector<rbmc_model*> owner;
  std::vector<int> np, nb;
  std::vector<const RegionDev*> rg;  // device pointers
  std::vector<int*> info;            // device flag per chain
  // block-Jacobi chains: S holds S_t^-1 for all T steps.  Subdomains: S holds
  // the forward inverses F_t = (S^f_t)^-1 for t < the last core step, G the
  // backward inverses G_t = (S^b_t)^-1 for t > the first core step (block
  // t - first core - 1), sig Sigma_tt of the first core step, sig2 that of the
  // core step in hand.
  std::vector<double*> S;
  std::vector<double*> G;
  std::vector<double*> tmp;          // np^2
  std::vector<double*> sig, sig2;    // np^2, subdomains only
  std::vector<double*> gjU, gjB;     // np x kSweepMax Gauss-Jordan panels
  std::vector<double*> gjP;          // kSweepMax^2 pivot block
  std::vector<double*> gjU2, gjB2;   // kSweepMax x 128 panels of the pivot block's sweep
  std::vector<double*> gjP2;         // 128 x 128
  // a second workspace set, for the backward inversion of the same round
  std::vector<double*> gjUb, gjBb, gjPb, gjU2b, gjB2b, gjP2b;
  std::vector<std::vector<double*>> pan;  // per chain: T panels np x n_k
  std::vector<double*> ytmp;              // per chain: one panel
  int maxT = 0;
  void append(const ChainSet& o) {
    auto cat = [](auto& a, const auto& b) { a.insert(a.end(), b.begin(), b.end()); };
    cat(chains, o.chains);
    cat(owner, o.owner);
    cat(np, o.np);
    cat(nb, o.nb);
    cat(rg, o.rg);
    cat(info, o.info);
    cat(S, o.S);
    cat(tmp, o.tmp);
    cat(G, o.G);
    cat(sig, o.sig);
    cat(sig2, o.sig2);
    cat(gjU, o.gjU);
    cat(gjB, o.gjB);
    cat(gjP, o.gjP);
    cat(gjU2, o.gjU2);
    cat(gjB2, o.gjB2);
    cat(gjUb, o.gjUb);
    cat(gjBb, o.gjBb);
    cat(gjPb, o.gjPb);
    cat(gjU2b, o.gjU2b);
    cat(gjB2b, o.gjB2b);
    cat(gjP2b, o.gjP2b);
    cat(gjP2, o.gjP2);
    cat(pan, o.pan);
    cat(ytmp, o.ytmp);
    maxT = std::max(maxT, o.maxT);
  }
  size_t size() const { return chains.size(); }
};

}  // namespace

struct rbmc_model {
  rbmc_ctx* ctx = nullptr;
  rbmc_model_desc desc{};
  std::vector<uint8_t> mask;
  rbmc_decomp_desc dc{};
  Plan plan;
  Coefs co;
  int n_obs = 0;
  Pool pool;      // model-lifetime allocations
  // chain sets are allocated on first use: the block-Jacobi chains by the
  // block-Jacobi preconditioner, the subdomain chains by the block-tridiagonal
  // method (at 512 x 512 x 48 either would exceed the device memory)
  bool bj_alloc = false, sub_alloc = false;
  Pool work_bj, work_sub;  // panels (sample-count dependent)
  int work_bj_nk = -1, work_sub_nk = -1;
  // Kronecker method: per subdomain, the observed slots grouped by local time
  // step (each group padded to a multiple of 16, the total to 64); per region,
  // S^-1 = (Q_s|R)^-1 and its node quantities
  struct KronSub {
    int chain = 0, TA = 0, nc = 0, nobs = 0;
    std::vector<int> goff, gpad;
    int *d_obs_a = nullptr, *d_obs_t = nullptr, *d_goff = nullptr, *d_gpad = nullptr;
  };
  struct KronReg {
    int region = 0, nb = 0, np = 0;
    double *inv = nullptr, *dR = nullptr, *qR = nullptr, *kR = nullptr;
    // rim of R: nodes with a 13-point neighbour in the grid outside R (the
    // only rows where r = Q_AB x_B is nonzero at steps away from the time
    // separator), nring of them, padded to nrp with -1; rinv = S^-1[:, rim]
    bool rim = false;  // corrections use the rim products
    int mc_win = 0;    // widest span of region rows the stencils of a 256-row chunk reach
    int nring = 0, nrp = 0;
    int* d_ring = nullptr;
    double* rinv = nullptr;
  };
  std::vector<KronSub> ksub;
  std::vector<KronReg> kreg;
  std::vector<int> kreg_of;  // plan region -> kreg index (-1: none)
  bool kron_static = false, kron_ready = false;
  Pool kpool;
  double* d_kk13 = nullptr;  // K in the 13-point layout (rows 5..12 zero)
  // spectral preconditioner data (allocated on first use)
  bool spec_alloc = false, spec_ready = false;
  double *d_lam = nullptr, *d_dctx = nullptr, *d_dcty = nullptr, *d_spcp = nullptr,
         *d_spid = nullptr, *d_spoff = nullptr;
  // transform route: 2 FFT (both sides powers of two), 1 matrix-core GEMM,
  // 0 the direct kernel; FFT twiddles (N/2 + N pairs per axis)
  int spec_route = 0;
  double *d_fftx = nullptr, *d_ffty = nullptr;
  Pool spool;
  DevModel dm{};
  DevModel* d_dm = nullptr;
  double *d_qs = nullptr, *d_kk = nullptr, *d_fs = nullptr, *d_qd = nullptr, *d_dqd = nullptr,
         *d_ld = nullptr, *d_dvec = nullptr;
  int* d_obs_rank = nullptr;
  uint32_t* d_obs_bits = nullptr;
  int* d_obs_wrank = nullptr;
  int* d_sep = nullptr;  // Alg. 2 separator nodes (plan.sep_nodes)
  std::vector<RegionDev> regions;
  RegionDev* d_regions = nullptr;
  ChainSet bj, sub;
  int* d_info = nullptr;  // one per chain: bj then sub
  bool bj_ready = false, sub_ready = false;
  // learned correction to the block-Jacobi preconditioner
  struct Learned {
    bool ready = false;          // weights present
    bool usable = false;         // validated: reduces the preconditioner error
    double val_rel_err = -1.0;   // held-out energy error with / without N_w
    int trial_bj = -1, trial_lrn = -1;  // PCG iterations of the acceptance trial
    double trial_s_bj = -1.0, trial_s_lrn = -1.0;  // and its sampler seconds
    float* w = nullptr;          // FP32 weights (device)
    uint16_t* wb = nullptr;      // BF16 weights used by the kernels
    uint16_t* wf = nullptr;      // BF16 flipped/transposed weights (input gradients)
    float *am = nullptr, *av = nullptr, *g = nullptr;  // Adam moments, gradient
  } lrn;
  Pool lwork;                    // inference activations
  size_t lwork_cols = 0;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

rbmc_status upload_coefs(rbmc_model* m) {
  const Plan& P = m->plan;
  const Coefs& c = m->co;
  hipStream_t s = m->ctx->stream;
  HIPCHK(hipMemcpyAsync(m->d_qs, c.qs.data(), c.qs.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m->d_kk, c.kk.data(), c.kk.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m->d_fs, c.fs.data(), c.fs.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m->d_qd, c.qd.data(), c.qd.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m->d_dqd, c.dqd.data(), c.dqd.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(m->d_ld, c.ld.data(), c.ld.size() * 8, hipMemcpyHostToDevice, s));
  std::vector<double> dv(P.n);
  for (int i = 0; i < P.n; ++i) dv[i] = m->mask[i] ? c.dobs : 0.0;
  HIPCHK(hipMemcpyAsync(m->d_dvec, dv.data(), dv.size() * 8, hipMemcpyHostToDevice, s));
  m->dm.qo = c.qo;
  m->dm.dqo = c.dqo;
  m->dm.lo = c.lo;
  m->dm.dobs = c.dobs;
  HIPCHK(hipMemcpyAsync(m->d_dm, &m->dm, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  m->bj_ready = m->sub_ready = false;
  m->kron_ready = false;
  m->spec_ready = false;
  return RBMC_OK;
}

bool theta_ok(double lk, double lt, double rho, double ls) {
  return std::isfinite(lk) && std::isfinite(lt) && std::isfinite(rho) && std::isfinite(ls) &&
         std::fabs(rho) < 1.0;
}

rbmc_status alloc_chainset(rbmc_model* m, ChainSet& cs, const std::vector<Chain>& chains,
                           bool subdomains, int info_base) {
  cs = ChainSet();
  for (size_t i = 0; i < chains.size(); ++i) {
    const Chain& c = chains[i];
    const int nb = m->plan.regions[c.region].nb();
    const int np = pad_to(nb);
    cs.chains.push_back(c);
    cs.owner.push_back(m);
    cs.np.push_back(np);
    cs.nb.push_back(nb);
    cs.rg.push_back(m->d_regions + c.region);
    cs.info.push_back(m->d_info + info_base + (int)i);
    const size_t blk = (size_t)np * np;
    double* p = nullptr;
    const int lc0 = c.ct0 - c.t0, lc1 = lc0 + c.cT - 1;
    const int nF = subdomains ? lc1 : c.T, nG = subdomains ? c.T - 1 - lc0 : 0;
    p = nullptr;
    if (nF > 0) HIPCHK(m->pool.alloc((void**)&p, blk * nF * 8));
    cs.S.push_back(p);
    p = nullptr;
    if (nG > 0) HIPCHK(m->pool.alloc((void**)&p, blk * nG * 8));
    cs.G.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, blk * 8));
    cs.tmp.push_back(p);
    if (subdomains) {
      HIPCHK(m->pool.alloc((void**)&p, blk * 8));
      cs.sig.push_back(p);
      HIPCHK(m->pool.alloc((void**)&p, blk * 8));
      cs.sig2.push_back(p);
    } else {
      cs.sig.push_back(nullptr);
      cs.sig2.push_back(nullptr);
    }
    const size_t wmax = sweep_width_of(np);  // widest step on this block
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * wmax * 8));
    cs.gjU.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * wmax * 8));
    cs.gjB.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * wmax * 8));
    cs.gjP.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * 128 * 8));
    cs.gjU2.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * 128 * 8));
    cs.gjB2.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)128 * 128 * 8));
    cs.gjP2.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * wmax * 8));
    cs.gjUb.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * wmax * 8));
    cs.gjBb.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * wmax * 8));
    cs.gjPb.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * 128 * 8));
    cs.gjU2b.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, wmax * 128 * 8));
    cs.gjB2b.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)128 * 128 * 8));
    cs.gjP2b.push_back(p);
    cs.pan.push_back({});
    cs.ytmp.push_back(nullptr);
    cs.maxT = std::max(cs.maxT, c.T);
  }
  return RBMC_OK;
}

// The block-Jacobi (bj) or subdomain chain set of a model, allocated on first
// use, with its correction / preconditioner panels for n_k samples.
rbmc_status ensure_chains(rbmc_model* m, bool bj, int n_k) {
  bool& done = bj ? m->bj_alloc : m->sub_alloc;
  ChainSet& cs = bj ? m->bj : m->sub;
  if (!done) {
    rbmc_status st = bj ? alloc_chainset(m, m->bj, m->plan.bj, false, 0)
                        : alloc_chainset(m, m->sub, m->plan.sub, true, (int)m->plan.bj.size());
    if (st != RBMC_OK) return st;
    done = true;
  }
  const int nk = std::max(n_k, 1);
  Pool& work = bj ? m->work_bj : m->work_sub;
  int& work_nk = bj ? m->work_bj_nk : m->work_sub_nk;
  if (work_nk >= nk) return RBMC_OK;
  work.release();
  work_nk = -1;
  for (size_t c = 0; c < cs.size(); ++c) {
    const size_t psz = (size_t)cs.np[c] * nk * 8;
    cs.pan[c].clear();
    for (int t = 0; t < cs.chains[c].T; ++t) {
      double* p = nullptr;
      HIPCHK(work.alloc((void**)&p, psz));
      cs.pan[c].push_back(p);
    }
    HIPCHK(work.alloc((void**)&cs.ytmp[c], psz));
  }
  work_nk = nk;
  return RBMC_OK;
}

// ---- task builders ----------------------------------------------------------

// A launch with fewer 128-tiles than this runs the 64 x 64-tile FP64 kernel
// (two workgroups per CU on 128-tiles would leave most of the device idle or
// latency-bound).

struct GemmList {
  std::vector<GemmTask> v;  // tile_start / tiles_n are set when the list is launched
  int mixed = 0;       // 1: FP32 matrix-core products, FP64 accumulation
  double flops = 0.0;  // algorithmic (unpadded) flops of the list
  double last_flops = 0.0;
  void add(const double* A, const double* B, const double* Cin, double* C, int M, int N, int K,
           int lda, int ldb, int ldc, double alpha, double beta, int tA, int tB, int Mreal,
           int Kreal) {
    last_flops = 2.0 * Mreal * (double)N * Kreal;
    flops += last_flops;
    GemmTask t{};
    t.A = A;
    t.B = B;
    t.Cin = Cin ? Cin : C;
    t.C = C;
    t.M = M;
    t.N = N;
    t.K = K;
    t.lda = lda;
    t.ldb = ldb;
    t.ldc = ldc;
    t.ldcin = ldc;
    t.alpha = alpha;
    t.beta = beta;
    t.transA = tA;
    t.transB = tB;
    v.push_back(t);
  }
  // restrict the last product to the lower tiles of a square result
  void set_last_lower() {
    GemmTask& t = v.back();
    flops -= 0.5 * last_flops;  // a symmetric result: the lower half is the work
    t.lower = 1;
  }
  // choose the kernel and number the tiles; returns the total tile count
  int finalize(int* kind) {
    int t128 = 0, kmax = 0;
    for (const GemmTask& t : v) {
      t128 += gemm_task_tiles(t.M, t.N, t.lower, 128);
      kmax = std::max(kmax, t.K);
    }
    // measured on MI355X: the 64-tile kernel is faster for short K (<= 256)
    // at any tile count, and whenever the 128-tiles would not fill the device
    *kind = mixed ? kGemmMixed
                  : ((t128 < g_tune.small_tiles || kmax <= g_tune.small_k) ? kGemmSmall : kGemmF64);
    const int ts = (*kind == kGemmSmall) ? 64 : 128;
    int tiles = 0;
    for (GemmTask& t : v) {
      t.tiles_n = (t.N + ts - 1) / ts;
      t.tile_start = tiles;
      tiles += gemm_task_tiles(t.M, t.N, t.lower, ts);
    }
    return tiles;
  }
  // outer sweep update of the lower tiles: M -= Ut^T Bt outside rows/cols
  // [kb, kb + w), with the transposed panels Ut, Bt (w x np, ld w)
  // (nb: unpadded size, for the algorithmic flops of the lower half)
  void add_sweep(double* Mx, int np, const double* Ut, const double* Bt, int w, int kb, int nb) {
    const double r = std::max(0, nb - w);
    flops += r * r * w;
    GemmTask t{};
    t.A = Ut;
    t.B = Bt;
    t.Cin = Mx;
    t.C = Mx;
    t.M = np;
    t.N = np;
    t.K = w;
    t.lda = w;
    t.ldb = w;
    t.ldc = np;
    t.ldcin = np;
    t.alpha = -1.0;
    t.beta = 1.0;
    t.transA = 1;
    t.transB = 0;
    t.lower = 1;
    t.skip0 = kb;
    t.skip1 = kb + w;
    v.push_back(t);
  }
};

struct StencilList {
  std::vector<StencilTask> v;
  int tiles = 0;
  double bytes = 0.0;
  int max_sparse_np = 0;  // largest block with sparse terms (0: none)
  int two = 0;            // some task has a second input M2
  void add(StencilTask t, int np, int nb) {
    t.tile_start = tiles;
    if (t.M2) two = 1;
    tiles += rstencil_tiles(np, t.ncols);
    bytes += 16.0 * nb * (double)t.ncols;
    if (t.gamma != 0.0 || t.dv != nullptr || t.pad_identity)
      max_sparse_np = std::max(max_sparse_np, np);
    v.push_back(t);
  }
};

template <class T>
struct TileList {
  std::vector<T> v;
  int tiles = 0;
  double bytes = 0.0;
  void add(T t, int ntiles, double b = 0.0) {
    t.tile_start = tiles;
    tiles += ntiles;
    bytes += b;
    v.push_back(t);
  }
};

struct InvJob {  // one SPD block to invert in place, with its workspace
  double* M;
  int np, nb;
  int* info;
  int base;            // row offset of M in the outermost block (for info)
  double *B, *U, *P;   // 256 x np, 256 x np, 256 x 256: transposed sweep panels, pivot block
  double *B2, *U2, *P2; // 128 x 256, 128 x 256, 128 x 128: the same one level down
};

struct Op {
  // 0 gemm, 1 stencil, 2 register inversion, 3 panels, 4 extract, 5 mc, 6 copy,
  // 7 outer gather, 8 outer fix, 9 sweep finish, 10 profile begin, 11 profile end, 12 mirror,
  // 13 off-diagonal pattern entries, 14-19 Kronecker-form kernels (region, build,
  // reduce, det, time mix, observed gather), 20 fill with zeros, 21 spectral
  // tridiagonal solves, 22 direct DCT along one axis, 23 FFT DCT along one axis
  int kind;
  size_t off = 0;
  int n = 0, tiles = 0;
  int max_np = 0, kblk = 0;
  void* dst = nullptr;
  const void* src = nullptr;
  size_t bytes = 0;
  int family = -1;
  double alg_flops = 0.0, alg_bytes = 0.0;
  ColSet cols{};  // kinds 21, 22
};

struct Program {
  std::vector<Op> ops;
  void gemm(Arena& a, GemmList& g, bool profiled = true, int family = -1) {
    if (g.v.empty()) return;
    Op o;
    o.kind = 0;
    o.tiles = g.finalize(&o.kblk);
    o.off = a.push(g.v);
    o.n = (int)g.v.size();
    o.family = !profiled ? -1
               : family >= 0 ? family
               : o.kblk == kGemmMixed ? RBMC_KF_GEMM_MIXED
               : o.kblk == kGemmSmall ? RBMC_KF_GEMM_SMALL : RBMC_KF_GEMM;
    o.alg_flops = g.flops;
    ops.push_back(o);
  }
  void stencil(Arena& a, StencilList& s) {
    if (s.v.empty()) return;
    Op o;
    o.kind = 1;
    o.off = a.push(s.v);
    o.n = (int)s.v.size();
    o.tiles = s.tiles;
    o.family = RBMC_KF_RSTENCIL;
    o.alg_bytes = s.bytes;
    o.max_np = s.max_sparse_np;
    o.kblk = s.two;
    ops.push_back(o);
  }
  void mirror(Arena& a, const std::vector<InvTask>& t) {
    if (t.empty()) return;
    Op o;
    o.kind = 12;
    o.off = a.push(t);
    o.n = (int)t.size();
    for (const InvTask& it : t) o.max_np = std::max(o.max_np, it.np);
    ops.push_back(o);
  }
  // register-resident inversion of blocks of order <= 128
  void inv128(Arena& a, const std::vector<SmallInvTask>& t) {
    if (t.empty()) return;
    Op o;
    o.kind = 2;
    o.off = a.push(t);
    o.n = (int)t.size();
    o.family = RBMC_KF_INV_SMALL;
    for (const SmallInvTask& k : t) o.alg_flops += (double)k.w * k.w * k.w;
    ops.push_back(o);
  }
  // In-place inversion of SPD blocks: blocks up to 128 in registers; larger
  // ones by outer sweeps of width w (GEMM updates of the lower tiles) whose
  // pivot blocks are inverted the same way one level down, then the finish
  // pass (negate and mirror).  Few blocks (a latency-bound chain) take w = 128
  // and a register inversion per step; many blocks take w = 256, halving the
  // passes of the rank-w updates over the blocks.
  void inverse(Arena& a, const std::vector<InvJob>& jobs) {
    if (jobs.empty()) return;
    Op pb;
    pb.kind = 10;
    pb.family = RBMC_KF_SPD_INVERSE;
    for (const InvJob& j : jobs) pb.alg_flops += (double)j.nb * j.nb * j.nb;
    ops.push_back(pb);
    int w = 128;
    if (jobs.size() >= 4) {
      w = kSweepMax;
      for (const InvJob& j : jobs) w = std::min(w, j.np >= g_tune.wide_from ? kSweepMax : 256);
    }
    sweep(a, jobs, w);
    Op pe;
    pe.kind = 11;
    ops.push_back(pe);
  }
  void sweep(Arena& a, const std::vector<InvJob>& jobs, int wo) {
    std::vector<SmallInvTask> small;
    std::vector<InvTask> big;
    int max_big = 0;
    for (const InvJob& j : jobs) {
      if (j.np <= 128) {
        small.push_back(SmallInvTask{j.M, j.np, j.np, j.info, j.base});
      } else {
        big.push_back(InvTask{j.M, j.np, j.nb, j.info});
        max_big = std::max(max_big, j.np);
      }
    }
    inv128(a, small);
    for (int kb = 0; kb < max_big; kb += wo) {
      TileList<Gj2Task> gl;
      std::vector<InvJob> inner;
      GemmList gu, gm;
      for (const InvJob& j : jobs) {
        if (j.np <= 128 || kb >= j.np) continue;
        const int w = std::min(wo, j.np - kb);
        Gj2Task g{};
        g.M = j.M;
        g.B = j.B;
        g.U = j.U;
        g.P = j.P;
        g.np = j.np;
        g.kb = kb;
        g.w = w;
        gl.add(g, gj2_tiles(j.np, w));
        // the pivot block, inverted one level down with the inner workspace
        InvJob in{};
        in.M = j.P;
        in.np = w;
        in.nb = w;
        in.info = j.info;
        in.base = j.base + kb;
        in.B = j.B2;
        in.U = j.U2;
        in.P = j.P2;
        inner.push_back(in);
        // Ut = P^-1 Bt (P^-1 symmetric, read through the transposed path)
        gu.add(j.P, j.B, nullptr, j.U, w, j.np, w, w, w, w, 1.0, 0.0, 1, 0, w, w);
        gm.add_sweep(j.M, j.np, j.U, j.B, w, kb, j.nb);
      }
      Op og;
      og.kind = 7;
      og.off = a.push(gl.v);
      og.n = (int)gl.v.size();
      og.tiles = gl.tiles;
      ops.push_back(og);
      sweep(a, inner, 128);
      gemm(a, gu);
      gemm(a, gm);
      Op of = og;
      of.kind = 8;
      ops.push_back(of);
    }
    if (!big.empty()) {
      Op f;
      f.kind = 9;
      f.off = a.push(big);
      f.n = (int)big.size();
      f.max_np = max_big;
      ops.push_back(f);
    }
  }
  void panels(Arena& a, TileList<PanelTask>& p) {
    if (p.v.empty()) return;
    Op o;
    o.kind = 3;
    o.off = a.push(p.v);
    o.n = (int)p.v.size();
    o.tiles = p.tiles;
    o.family = RBMC_KF_PANELS;
    o.alg_bytes = p.bytes;
    ops.push_back(o);
  }
  void extract(Arena& a, TileList<ExtractTask>& e) {
    if (e.v.empty()) return;
    Op o;
    o.kind = 4;
    o.off = a.push(e.v);
    o.n = (int)e.v.size();
    o.tiles = e.tiles;
    ops.push_back(o);
  }
  void mc(Arena& a, TileList<McTask>& e, bool multi = false) {
    if (e.v.empty()) return;
    Op o;
    o.kind = 5;
    o.off = a.push(e.v);
    o.n = (int)e.v.size();
    o.tiles = e.tiles;
    o.kblk = multi ? 1 : 0;
    o.family = RBMC_KF_MC;
    o.alg_bytes = e.bytes;
    ops.push_back(o);
  }
  void offdiag(Arena& a, TileList<OffdiagTask>& t) {
    if (t.v.empty()) return;
    Op o;
    o.kind = 13;
    o.off = a.push(t.v);
    o.n = (int)t.v.size();
    o.tiles = t.tiles;
    o.family = RBMC_KF_OFFDIAG;
    o.alg_bytes = t.bytes;
    ops.push_back(o);
  }
  // Kronecker-form kernels (kinds 14-19)
  template <class T>
  void kron(Arena& a, int kind, TileList<T>& t, int family = -1) {
    if (t.v.empty()) return;
    Op o;
    o.kind = kind;
    o.off = a.push(t.v);
    o.n = (int)t.v.size();
    o.tiles = t.tiles;
    o.family = family;
    o.alg_bytes = t.bytes;
    ops.push_back(o);
  }
  void fill(double* p, size_t n) {
    if (n == 0) return;
    Op o;
    o.kind = 20;
    o.dst = p;
    o.bytes = n;
    ops.push_back(o);
  }
  void copy(void* dst, const void* src, size_t bytes) {
    Op o;
    o.kind = 6;
    o.dst = dst;
    o.src = src;
    o.bytes = bytes;
    ops.push_back(o);
  }
};

rbmc_status run(rbmc_ctx* cx, const Program& pg, hipStream_t s, Arena& a) {
  std::vector<int> open_prof;  // records opened by profile-begin ops
  for (const Op& o : pg.ops) {
    const int pid = (o.family >= 0) ? cx->begin(o.family, o.alg_flops, o.alg_bytes, s) : -1;
    switch (o.kind) {
      case 0:
        launch_gemm(a.at<GemmTask>(o.off), o.n, o.tiles, s, o.kblk,
                    o.family == RBMC_KF_DCT ? 1 : 0);
        break;
      case 1: launch_rstencil(a.at<StencilTask>(o.off), o.n, o.tiles, o.max_np, o.kblk, s); break;
      case 2: launch_inv128(a.at<SmallInvTask>(o.off), o.n, s); break;
      case 3: launch_panels(a.at<PanelTask>(o.off), o.n, o.tiles, s); break;
      case 4: launch_extract(a.at<ExtractTask>(o.off), o.n, o.tiles, s); break;
      case 5: launch_mc(a.at<McTask>(o.off), o.n, o.tiles, o.kblk, s); break;
      case 6: HIPCHK(hipMemcpyAsync(o.dst, o.src, o.bytes, hipMemcpyDeviceToDevice, s)); break;
      case 7: launch_gj2_gather(a.at<Gj2Task>(o.off), o.n, o.tiles, s); break;
      case 8: launch_gj2_fix(a.at<Gj2Task>(o.off), o.n, o.tiles, s); break;
      case 9: launch_gj_finish(a.at<InvTask>(o.off), o.n, o.max_np, s); break;
      case 10: open_prof.push_back(pid); break;
      case 11:
        if (!open_prof.empty()) {
          cx->end(open_prof.back(), s);
          open_prof.pop_back();
        }
        break;
      case 12: launch_mirror(a.at<InvTask>(o.off), o.n, o.max_np, s); break;
      case 13: launch_offdiag(a.at<OffdiagTask>(o.off), o.n, o.tiles, s); break;
      case 14: launch_kron_region(a.at<KronRegionTask>(o.off), o.n, o.tiles, s); break;
      case 15: launch_kron_build(a.at<KronBuildTask>(o.off), o.n, o.tiles, s); break;
      case 16: launch_kron_reduce(a.at<KronReduceTask>(o.off), o.n, o.tiles, s); break;
      case 17: launch_kron_det(a.at<KronDetTask>(o.off), o.n, o.tiles, s); break;
      case 18: launch_kron_tmix(a.at<KronMixTask>(o.off), o.n, o.tiles, s); break;
      case 19: launch_kron_obs(a.at<KronObsTask>(o.off), o.n, o.tiles, s); break;
      case 20: launch_fill((double*)o.dst, o.bytes, 0.0, s); break;
      case 21: launch_spec_solve(o.cols, (double*)o.dst, s); break;
      case 22: launch_dct_direct(o.cols, (const double*)o.src, (double*)o.dst, o.n, o.kblk, s); break;
      case 23: launch_dct_fft(a.at<FftTask>(o.off), o.n, o.tiles, o.kblk, o.max_np, s); break;
    }
    if (o.kind != 10) cx->end(pid, s);
  }
  HIPCHK(hipGetLastError());
  return RBMC_OK;
}

StencilTask stask(const ChainSet& cs, size_t c) {
  StencilTask t{};
  t.rg = cs.rg[c];
  t.qs = cs.owner[c]->d_qs;
  t.ns = cs.owner[c]->plan.ns;
  return t;
}


// Local core range [lc0, lc1] of a chain and its two-sided factor blocks.
// Subdomain chains: forward inverses F_t for t < lc1 in S, backward G_t for
// t > lc0 in G, Sigma at the first core step in sig.  Block-Jacobi chains
// (bj): twist k = T/2, F_t (t < k), Sigma_k and G_t (t > k) all in S at their
// step index.
inline int chain_lc0(const Chain& ch) { return ch.ct0 - ch.t0; }
inline int chain_lc1(const Chain& ch) { return ch.ct0 - ch.t0 + ch.cT - 1; }
inline int twist_of(const Chain& ch, bool bj) { return bj ? ch.T / 2 : chain_lc0(ch); }
inline int fwd_count(const Chain& ch, bool bj) { return bj ? ch.T / 2 : chain_lc1(ch); }
inline double* fblock(const ChainSet& cs, size_t c, int t) {
  return cs.S[c] + (size_t)cs.np[c] * cs.np[c] * t;
}
inline double* gblock(const ChainSet& cs, size_t c, int t, bool bj = false) {
  if (bj) return cs.S[c] + (size_t)cs.np[c] * cs.np[c] * t;
  return cs.G[c] + (size_t)cs.np[c] * cs.np[c] * (t - chain_lc0(cs.chains[c]) - 1);
}
inline double* sigblock(const ChainSet& cs, size_t c, bool bj) {
  return bj ? cs.S[c] + (size_t)cs.np[c] * cs.np[c] * (cs.chains[c].T / 2) : cs.sig[c];
}

// Stencil tasks forming  out = B_t - q_o^2 Q_R (X + Y) Q_R  (X, Y symmetric
// inverse blocks, either may be null; B_t = q_d(t) Q_R + D_t, identity on the
// padded diagonal) in two passes through cs.tmp[c]: tmp = (Q_R (X + Y))^T
// (stored transposed, i.e. (X + Y) Q_R; the sum is formed as the inputs are
// loaded), out = -q_o^2 Q_R tmp + B_t.
void add_schur(const ChainSet& cs, size_t c, int t, const double* X, const double* Y,
               double* out, StencilList& v1, StencilList& v2) {
  const Chain& ch = cs.chains[c];
  const rbmc_model* m = cs.owner[c];
  const int np = cs.np[c], nb = cs.nb[c];
  const int tg = ch.t0 + t;
  const double* first = X ? X : Y;
  const double* second = X ? Y : nullptr;
  if (first) {
    StencilTask s1 = stask(cs, c);
    s1.M = first;
    s1.M2 = second;
    s1.ldm = np;
    s1.out = cs.tmp[c];
    s1.ldout = np;
    s1.ncols = np;
    s1.alpha = 1.0;
    s1.tstore = 1;
    v1.add(s1, np, nb);
    if (second) v1.bytes += 8.0 * nb * (double)np;  // the second input's reads
  }
  StencilTask s2 = stask(cs, c);
  s2.M = first ? cs.tmp[c] : nullptr;
  s2.ldm = np;
  s2.alpha = first ? -m->co.qo * m->co.qo : 0.0;
  s2.gamma = m->co.qd[tg];
  s2.dv = m->d_dvec + (size_t)tg * m->plan.ns;
  s2.pad_identity = 1;
  s2.out = out;
  s2.ldout = np;
  s2.ncols = np;
  v2.add(s2, np, nb);
}

// ws: workspace set 0 or 1 (two inversions of one chain may share a batch)
InvJob inv_job(const ChainSet& cs, size_t c, double* M, int ws = 0) {
  InvJob it{};
  it.M = M;
  it.np = cs.np[c];
  it.nb = cs.nb[c];
  it.info = cs.info[c];
  it.B = ws ? cs.gjBb[c] : cs.gjB[c];
  it.U = ws ? cs.gjUb[c] : cs.gjU[c];
  it.P = ws ? cs.gjPb[c] : cs.gjP[c];
  it.B2 = ws ? cs.gjB2b[c] : cs.gjB2[c];
  it.U2 = ws ? cs.gjU2b[c] : cs.gjU2[c];
  it.P2 = ws ? cs.gjP2b[c] : cs.gjP2[c];
  it.base = 0;
  return it;
}

// Two-sided factorization of block-tridiagonal chains (diagonal blocks B_t,
// off-diagonal blocks q_o Q_R):
//   forward  F_0 = B_0^-1,      F_t = (B_t - q_o^2 Q_R F_{t-1} Q_R)^-1;
//   backward G_{T-1} = B_{T-1}^-1, G_t = (B_t - q_o^2 Q_R G_{t+1} Q_R)^-1.
// Subdomains: F for t < lc1, G for t > lc0 (their Sigma_tt are formed per
// call by the core-step program).  Block-Jacobi chains (bj): F for t < k,
// G for t > k and Sigma_k = (B_k - q_o^2 Q_R (F_{k-1} + G_{k+1}) Q_R)^-1 at the
// twist k = T/2, so the dependent chain of inversions is about half as long.
// Round r takes forward step r and backward step T-1-r of every chain: their
// stencil passes one after the other (they share cs.tmp), their inversions
// in one batch (each with its own workspace set).
void build_twosided(ChainSet& cs, Program& pg, Arena& a, bool bj = false) {
  int rounds = 0;
  for (size_t c = 0; c < cs.size(); ++c) {
    const Chain& ch = cs.chains[c];
    const int k0 = bj ? ch.T / 2 : chain_lc0(ch);
    rounds = std::max(rounds, std::max(fwd_count(ch, bj), ch.T - 1 - k0));
  }
  for (int r = 0; r < rounds; ++r) {
    std::vector<InvJob> inv;
    for (int dir = 0; dir < 2; ++dir) {
      StencilList v1, v2;
      for (size_t c = 0; c < cs.size(); ++c) {
        const Chain& ch = cs.chains[c];
        if (dir == 0) {
          if (r >= fwd_count(ch, bj)) continue;
          double* out = fblock(cs, c, r);
          add_schur(cs, c, r, r > 0 ? fblock(cs, c, r - 1) : nullptr, nullptr, out, v1, v2);
          inv.push_back(inv_job(cs, c, out));
        } else {
          const int t = ch.T - 1 - r;
          if (t <= (bj ? ch.T / 2 : chain_lc0(ch))) continue;
          double* out = gblock(cs, c, t, bj);
          add_schur(cs, c, t, t < ch.T - 1 ? gblock(cs, c, t + 1, bj) : nullptr, nullptr, out,
                    v1, v2);
          inv.push_back(inv_job(cs, c, out, 1));
        }
      }
      pg.stencil(a, v1);
      pg.stencil(a, v2);
    }
    pg.inverse(a, inv);
  }
  if (bj) {  // Sigma at the twist
    StencilList v1, v2;
    std::vector<InvJob> inv;
    for (size_t c = 0; c < cs.size(); ++c) {
      const Chain& ch = cs.chains[c];
      const int k = ch.T / 2;
      double* out = sigblock(cs, c, true);
      add_schur(cs, c, k, k >= 1 ? fblock(cs, c, k - 1) : nullptr,
                k + 1 < ch.T ? gblock(cs, c, k + 1, true) : nullptr, out, v1, v2);
      inv.push_back(inv_job(cs, c, out));
    }
    pg.stencil(a, v1);
    pg.stencil(a, v2);
    pg.inverse(a, inv);
  }
}

// Twisted block solve Q_AA mu = r with the two-sided factors, meeting at the
// first core step k = lc0 (r_t in pan[c][t] for every t; cs.ytmp[c] and
// cs.tmp[c] are the work panels):
//   forward  u_t = F_t (r_t - q_o Q_R u_{t-1}),             t < k;
//   backward v_t = G_t (r_t - q_o Q_R v_{t+1}),             t > k;
//   twist    mu_k = Sigma_kk (r_k - q_o Q_R u_{k-1} - q_o Q_R v_{k+1});
//   then     mu_{k-1} = u_{k-1} - F_{k-1} q_o Q_R mu_k,
//            mu_t = v_t - G_t q_o Q_R mu_{t-1}   for k < t <= lc1 + 1,
// i.e. mu on every step the Monte Carlo terms of the core rows read.  Block-
// Jacobi chains (bj): twist k = T/2 and the back substitution runs over the
// whole chain (the preconditioned residual).
void build_twisted_solve(ChainSet& cs, int n_k, Program& pg, Arena& a, int mixed,
                         bool bj = false) {
  // Work panels: ytmp for the forward (downward) direction; for the backward
  // (upward) one the chain's Schur temporary, idle during the solves, when
  // n_k <= np, so both directions of a round share one stencil and one GEMM
  // launch.  Otherwise the directions take turns with ytmp.
  bool pair = true;
  for (size_t c = 0; c < cs.size(); ++c) pair = pair && n_k <= cs.np[c];
  auto work = [&](size_t c, int dir) { return (dir == 1 && pair) ? cs.tmp[c] : cs.ytmp[c]; };
  auto stencil_into = [&](size_t c, double* y, const double* M, double alpha, const double* In,
                          StencilList& sl) {
    StencilTask st = stask(cs, c);
    st.M = M;
    st.ldm = cs.np[c];
    st.alpha = M ? alpha : 0.0;
    st.In = In;
    st.ldin = cs.np[c];
    st.beta = In ? 1.0 : 0.0;
    st.out = y;
    st.ldout = cs.np[c];
    st.ncols = n_k;
    sl.add(st, cs.np[c], cs.nb[c]);
  };
  auto gemm = [&](size_t c, const double* y, const double* Sinv, const double* Cin, double* C,
                  double alpha, double beta, GemmList& gl) {
    const int np = cs.np[c], nb = cs.nb[c];
    gl.add(Sinv, y, Cin, C, np, n_k, np, np, np, np, alpha, beta, 1, 0, nb, nb);
  };
  // one round: list 0 holds both directions when paired, else list dir
  auto emit = [&](StencilList* sl, GemmList* gl) {
    for (int dir = 0; dir < 2; ++dir) {
      pg.stencil(a, sl[dir]);
      pg.gemm(a, gl[dir]);
    }
  };
  for (int t = 0; t < cs.maxT; ++t) {  // forward and backward partial solutions
    StencilList sl[2];
    GemmList gl[2];
    gl[0].mixed = gl[1].mixed = mixed;
    for (int dir = 0; dir < 2; ++dir) {
      const int li = pair ? 0 : dir;
      for (size_t c = 0; c < cs.size(); ++c) {
        const Chain& ch = cs.chains[c];
        const double qo = cs.owner[c]->co.qo;
        const int k = twist_of(ch, bj);
        double* y = work(c, dir);
        if (dir == 0) {
          if (t >= k) continue;
          stencil_into(c, y, t > 0 ? cs.pan[c][t - 1] : nullptr, -qo, cs.pan[c][t], sl[li]);
          gemm(c, y, fblock(cs, c, t), nullptr, cs.pan[c][t], 1.0, 0.0, gl[li]);
        } else {
          const int tt = ch.T - 1 - t;
          if (tt <= k) continue;
          stencil_into(c, y, tt < ch.T - 1 ? cs.pan[c][tt + 1] : nullptr, -qo, cs.pan[c][tt],
                       sl[li]);
          gemm(c, y, gblock(cs, c, tt, bj), nullptr, cs.pan[c][tt], 1.0, 0.0, gl[li]);
        }
      }
    }
    emit(sl, gl);
  }
  {  // twist
    StencilList s1, s2;
    GemmList gl;
    gl.mixed = mixed;
    for (size_t c = 0; c < cs.size(); ++c) {
      const Chain& ch = cs.chains[c];
      const double qo = cs.owner[c]->co.qo;
      const int k = twist_of(ch, bj);
      double* y = cs.ytmp[c];
      stencil_into(c, y, k > 0 ? cs.pan[c][k - 1] : nullptr, -qo, cs.pan[c][k], s1);
      if (k + 1 < ch.T) stencil_into(c, y, cs.pan[c][k + 1], -qo, y, s2);
      gemm(c, y, sigblock(cs, c, bj), nullptr, cs.pan[c][k], 1.0, 0.0, gl);
    }
    pg.stencil(a, s1);
    pg.stencil(a, s2);
    pg.gemm(a, gl);
  }
  // outward: subdomains one step below the core and up to one above it;
  // block-Jacobi chains down to step 0 and up to T-1 (the down and up steps
  // of the same distance form one round)
  for (int d = 1; d < cs.maxT; ++d) {
    StencilList sl[2];
    GemmList gl[2];
    gl[0].mixed = gl[1].mixed = mixed;
    for (int dir = 0; dir < 2; ++dir) {
      const int li = pair ? 0 : dir;
      for (size_t c = 0; c < cs.size(); ++c) {
        const Chain& ch = cs.chains[c];
        const int k = twist_of(ch, bj);
        const double qo = cs.owner[c]->co.qo;
        double* y = work(c, dir);
        if (dir == 0) {
          const int t = k - d;
          if (t < 0 || (!bj && d > 1)) continue;
          stencil_into(c, y, cs.pan[c][t + 1], qo, nullptr, sl[li]);
          gemm(c, y, fblock(cs, c, t), cs.pan[c][t], cs.pan[c][t], -1.0, 1.0, gl[li]);
        } else {
          const int t = k + d;
          if (t >= ch.T || (!bj && t > chain_lc1(ch) + 1)) continue;
          stencil_into(c, y, cs.pan[c][t - 1], qo, nullptr, sl[li]);
          gemm(c, y, gblock(cs, c, t, bj), cs.pan[c][t], cs.pan[c][t], -1.0, 1.0, gl[li]);
        }
      }
    }
    emit(sl, gl);
  }
}


rbmc_status check_info(const ChainSet& cs, rbmc_report* rep, const char* what, hipStream_t s) {
  for (size_t c = 0; c < cs.size(); ++c) {
    int v = 0;
    HIPCHK(hipMemcpyAsync(&v, cs.info[c], 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (v != 0) {
      if (rep) {
        rep->fail_subdomain = (int)c;
        rep->fail_block = v - 1;
      }
      return fail(RBMC_E_NOT_SPD, std::string(what) + " chain " + std::to_string(c) +
                                      " lost positive definiteness");
    }
  }
  return RBMC_OK;
}

rbmc_status zero_info(const ChainSet& cs, hipStream_t s) {
  for (size_t c = 0; c < cs.size(); ++c) HIPCHK(hipMemsetAsync(cs.info[c], 0, 4, s));
  return RBMC_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void init_report(rbmc_report* rep) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  rep->fail_subdomain = -1;
  rep->fail_block = -1;
}

rbmc_status check_opts(const rbmc_est_opts* o, bool need_pcg) {
  if (!o) return fail(RBMC_E_ARG, "opts is NULL");
  if (o->n_samples < 0) return fail(RBMC_E_ARG, "n_samples must be >= 0");
  if (need_pcg && (o->pcg_maxit < 1 || !(o->pcg_rtol > 0.0)))
    return fail(RBMC_E_ARG, "pcg_maxit must be >= 1 and pcg_rtol > 0");
  if (o->grad_mask & ~15u) return fail(RBMC_E_ARG, "grad_mask has unknown bits");
  if (o->precision != RBMC_FP64 && o->precision != RBMC_MIXED)
    return fail(RBMC_E_ARG, "precision must be RBMC_FP64 or RBMC_MIXED");
  if (o->precond != RBMC_PC_BJ && o->precond != RBMC_PC_BJ_LEARNED &&
      o->precond != RBMC_PC_SPECTRAL)
    return fail(RBMC_E_ARG, "precond must be RBMC_PC_BJ, RBMC_PC_BJ_LEARNED or RBMC_PC_SPECTRAL");
  if (o->method != RBMC_SEL_AUTO && o->method != RBMC_SEL_BLOCKTRI && o->method != RBMC_SEL_KRON)
    return fail(RBMC_E_ARG, "method must be RBMC_SEL_AUTO, RBMC_SEL_BLOCKTRI or RBMC_SEL_KRON");
  if (o->sample_chunk < 0) return fail(RBMC_E_ARG, "sample_chunk must be >= 0");
  return RBMC_OK;
}

// ---------------------------------------------------------------------------
// Column sets of the sampler: columns (model j, sample k), model-major.
// Column (j, k) of a multi-vector starts at base_j + k n_j with base_j the
// sum of n_i n_k over earlier models; the F input column at
// zbase_j + k (n_j + n_obs_j).
// ---------------------------------------------------------------------------
struct HostCols {
  std::vector<int64_t> off, in_off;
  std::vector<int> len, model;
  std::vector<size_t> base, zbase;  // per model
  size_t total = 0, ztotal = 0;
  int max_len = 0, max_tiles = 0, max_ns = 0, max_T = 0;
};

// kernels over columns put the column index in grid.y
constexpr int64_t kMaxCols = 65535;

bool cols_fit(size_t n_models, int nk) { return (int64_t)n_models * nk <= kMaxCols; }

HostCols make_cols(const std::vector<rbmc_model*>& ms, int nk) {
  HostCols h;
  for (size_t j = 0; j < ms.size(); ++j) {
    const rbmc_model* m = ms[j];
    h.base.push_back(h.total);
    h.zbase.push_back(h.ztotal);
    for (int k = 0; k < nk; ++k) {
      h.off.push_back((int64_t)(h.total + (size_t)k * m->plan.n));
      h.in_off.push_back((int64_t)(h.ztotal + (size_t)k * (m->plan.n + m->n_obs)));
      h.len.push_back(m->plan.n);
      h.model.push_back((int)j);
    }
    h.total += (size_t)m->plan.n * nk;
    h.ztotal += (size_t)(m->plan.n + m->n_obs) * nk;
    h.max_len = std::max(h.max_len, m->plan.n);
    h.max_ns = std::max(h.max_ns, m->plan.ns);
    h.max_T = std::max(h.max_T, m->plan.T);
    h.max_tiles = std::max(h.max_tiles, stencil_tiles(m->plan.mx, m->plan.my));
  }
  return h;
}

// Sampler workspace of the context for a column set (grown on demand).
rbmc_status ensure_ws(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, const HostCols& h,
                      bool need_zcat) {
  const int ncols = (int)h.len.size();
  const size_t part = (size_t)std::max(1, ncols) *
                      (size_t)std::max(h.max_tiles, dot_chunks(std::max(h.max_len, 1)));
  const bool fits = cx->ws_len >= h.total && cx->ws_cols >= ncols && cx->part_len >= part &&
                    cx->ws_models >= (int)ms.size() && (!need_zcat || cx->ws_zlen >= h.ztotal);
  if (!fits) {
    cx->ws.release();
    cx->ws_len = cx->ws_zlen = 0;
    cx->ws_cols = cx->ws_models = 0;
    cx->zcat = nullptr;
    const size_t len = std::max<size_t>(h.total, 1);
    // the Kronecker workspace holds nothing between its batches (each ends
    // synchronized): give it up when the sampler's vectors would not fit
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const size_t need = (6 * len + (need_zcat ? h.ztotal : 0)) * 8 + ((size_t)1 << 30);
    if (fr < need && cx->kws_cap > 0) {
      cx->kws.release();
      cx->kws_base = nullptr;
      cx->kws_cap = 0;
    }
    HIPCHK(cx->ws.alloc((void**)&cx->r, len * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->p, len * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->q, len * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->z, len * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->x, len * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->zp, len * 8));
    if (need_zcat) {
      HIPCHK(cx->ws.alloc((void**)&cx->zcat, std::max<size_t>(h.ztotal, 1) * 8));
      cx->ws_zlen = h.ztotal;
    }
    const int nc = std::max(ncols, 1);
    HIPCHK(cx->ws.alloc((void**)&cx->scal, (size_t)9 * nc * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->part, part * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->active, (size_t)nc));
    HIPCHK(cx->ws.alloc((void**)&cx->iters, (size_t)(nc + 1) * 4));
    HIPCHK(cx->ws.alloc((void**)&cx->d_off, (size_t)nc * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->d_in_off, (size_t)nc * 8));
    HIPCHK(cx->ws.alloc((void**)&cx->d_len, (size_t)nc * 4));
    HIPCHK(cx->ws.alloc((void**)&cx->d_model, (size_t)nc * 4));
    HIPCHK(cx->ws.alloc((void**)&cx->d_dms, std::max<size_t>(ms.size(), 1) * sizeof(DevModel)));
    cx->ws_len = h.total;
    cx->ws_cols = ncols;
    cx->part_len = part;
    cx->ws_models = (int)ms.size();
  }
  hipStream_t s = cx->stream;
  const int nc = ncols;
  if (nc > 0) {
    HIPCHK(hipMemcpyAsync(cx->d_off, h.off.data(), (size_t)nc * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cx->d_in_off, h.in_off.data(), (size_t)nc * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cx->d_len, h.len.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cx->d_model, h.model.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s));
  }
  std::vector<DevModel> dms;
  for (rbmc_model* m : ms) dms.push_back(m->dm);
  if (!dms.empty())
    HIPCHK(hipMemcpyAsync(cx->d_dms, dms.data(), dms.size() * sizeof(DevModel),
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBMC_OK;
}

ColSet colset(rbmc_ctx* cx, const HostCols& h) {
  ColSet c{};
  c.ncols = (int)h.len.size();
  c.max_len = h.max_len;
  c.max_tiles = h.max_tiles;
  c.max_ns = h.max_ns;
  c.max_T = h.max_T;
  c.off = cx->d_off;
  c.in_off = cx->d_in_off;
  c.len = cx->d_len;
  c.model = cx->d_model;
  c.dms = cx->d_dms;
  return c;
}

// ---------------------------------------------------------------------------
// Spectral preconditioner M = Q_t (x) Q_s + dbar I.  The orthonormal DCT-II
// matrix C (C[k, i] = c_k cos(pi k (2 i + 1) / (2 m)), c_0 = m^-1/2, else
// (2/m)^1/2) diagonalizes the Neumann path Laplacian, C G_1 C^T = diag(2 - 2
// cos(pi k / m)), so the 2-D transform diagonalizes G = G_x (+) G_y and every
// polynomial in it: Q_s = tau (kappa^4 h^2 I + 2 kappa^2 G + G^2 / h^2) has
// eigenvalue lambda_f = tau (kappa^4 h^2 + 2 kappa^2 l + l^2 / h^2) at
// frequency f = (kx, ky), l = l_x(kx) + l_y(ky).  In that basis M is one
// tridiagonal system per frequency (lambda_f Q_t + dbar I).
// ---------------------------------------------------------------------------
void dct_matrix(int m, std::vector<double>& C) {
  C.assign((size_t)m * m, 0.0);
  for (int k = 0; k < m; ++k) {
    const double ck = k == 0 ? std::sqrt(1.0 / m) : std::sqrt(2.0 / m);
    for (int i = 0; i < m; ++i) C[(size_t)i * m + k] = ck * std::cos(M_PI * k * (2 * i + 1) / (2.0 * m));
  }
}

rbmc_status upload_dm(rbmc_model* m, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(m->d_dm, &m->dm, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBMC_OK;
}

rbmc_status ensure_spectral(rbmc_model* m, hipStream_t s) {
  const Plan& P = m->plan;
  if (!m->spec_alloc) {
    const bool fft_ok = fft_length_ok(P.mx) && fft_length_ok(P.my);
    const bool gemm_ok = P.mx % 16 == 0 && P.my % 16 == 0 && P.mx >= 64 && P.my >= 64;
    m->spec_route = fft_ok ? 2 : gemm_ok ? 1 : 0;
    if (const char* e = std::getenv("RBMC_SPEC_ROUTE")) {  // "fft", "gemm" or "direct"
      const std::string r(e);
      if (r == "direct") m->spec_route = 0;
      if (r == "gemm" && gemm_ok) m->spec_route = 1;
      if (r == "fft" && fft_ok) m->spec_route = 2;
    }
    if (m->spec_route == 2) {
      for (int ax = 0; ax < 2; ++ax) {
        const int N = ax == 0 ? P.mx : P.my;
        std::vector<double> tab((size_t)3 * N);  // tw (N/2 pairs), then ph (N pairs)
        for (int t = 0; t < N / 2; ++t) {
          tab[2 * t] = std::cos(2.0 * M_PI * t / N);
          tab[2 * t + 1] = std::sin(2.0 * M_PI * t / N);
        }
        for (int k = 0; k < N; ++k) {
          tab[N + 2 * k] = std::cos(M_PI * k / (2.0 * N));
          tab[N + 2 * k + 1] = std::sin(M_PI * k / (2.0 * N));
        }
        double*& d = ax == 0 ? m->d_fftx : m->d_ffty;
        HIPCHK(m->spool.alloc((void**)&d, tab.size() * 8));
        HIPCHK(hipMemcpyAsync(d, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // tab is host memory of this scope
      }
    }
    HIPCHK(m->spool.alloc((void**)&m->d_lam, (size_t)P.ns * 8));
    HIPCHK(m->spool.alloc((void**)&m->d_spoff, (size_t)P.ns * 8));
    HIPCHK(m->spool.alloc((void**)&m->d_spcp, (size_t)P.n * 8));
    HIPCHK(m->spool.alloc((void**)&m->d_spid, (size_t)P.n * 8));
    HIPCHK(m->spool.alloc((void**)&m->d_dctx, (size_t)P.mx * P.mx * 8));
    HIPCHK(m->spool.alloc((void**)&m->d_dcty, (size_t)P.my * P.my * 8));
    std::vector<double> C;
    dct_matrix(P.mx, C);
    HIPCHK(hipMemcpyAsync(m->d_dctx, C.data(), C.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    dct_matrix(P.my, C);
    HIPCHK(hipMemcpyAsync(m->d_dcty, C.data(), C.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    m->spec_alloc = true;
  }
  if (m->spec_ready) return RBMC_OK;
  const Coefs& co = m->co;
  const double k2 = co.kappa * co.kappa, h2 = co.h * co.h;
  std::vector<double> lx(P.mx), ly(P.my), lam((size_t)P.ns);
  for (int k = 0; k < P.mx; ++k) lx[k] = 2.0 - 2.0 * std::cos(M_PI * k / P.mx);
  for (int k = 0; k < P.my; ++k) ly[k] = 2.0 - 2.0 * std::cos(M_PI * k / P.my);
  for (int ky = 0; ky < P.my; ++ky)
    for (int kx = 0; kx < P.mx; ++kx) {
      const double l = lx[kx] + ly[ky];
      lam[(size_t)ky * P.mx + kx] = co.tau * (k2 * k2 * h2 + 2.0 * k2 * l + l * l / h2);
    }
  HIPCHK(hipMemcpyAsync(m->d_lam, lam.data(), lam.size() * 8, hipMemcpyHostToDevice, s));
  SpecCoefTask t{};
  t.lam = m->d_lam;
  t.qd = m->d_qd;
  t.qo = co.qo;
  t.dbar = P.n > 0 ? (double)m->n_obs * co.dobs / P.n : 0.0;
  t.ns = P.ns;
  t.T = P.T;
  t.cp = m->d_spcp;
  t.id = m->d_spid;
  t.off = m->d_spoff;
  launch_spec_coef(t, s);
  HIPCHK(hipGetLastError());
  m->dm.dct_x = m->d_dctx;
  m->dm.dct_y = m->d_dcty;
  m->dm.sp_cp = m->d_spcp;
  m->dm.sp_id = m->d_spid;
  m->dm.sp_off = m->d_spoff;
  m->dm.spec_gemm = m->spec_route != 0 ? 1 : 0;
  rbmc_status st = upload_dm(m, s);  // synchronizes: lam is on the host stack
  if (st != RBMC_OK) return st;
  m->spec_ready = true;
  return RBMC_OK;
}

// One axis of the 2-D transform for every column of the set: models with the
// FFT route by the FFT kernel (axis 0: the contiguous lines of length mx;
// axis 1: lines of length my, mx apart), models with the GEMM route as
// matrix-core products (axis 0: C_x X over all rows of x at once; axis 1:
// X_s C_y^T per (time step, sample) slice), the others by the direct
// kernel.  inverse: C^T.
void spectral_axis(const std::vector<rbmc_model*>& ms, const HostCols& h, const ColSet& cols,
                   int nk, const double* in, double* out, int axis, int inverse, Program& pg,
                   Arena& a) {
  GemmList gl;
  std::vector<FftTask> ft;
  int fft_tiles_total = 0;
  double fft_bytes = 0.0;
  bool direct = false;
  for (size_t j = 0; j < ms.size(); ++j) {
    const rbmc_model* m = ms[j];
    const int mx = m->plan.mx, my = m->plan.my, T = m->plan.T;
    if (!m->dm.spec_gemm) {
      direct = true;
      continue;
    }
    const double* src = in + h.base[j];
    double* dst = out + h.base[j];
    if (m->spec_route == 2) {
      FftTask t{};
      t.in = src;
      t.out = dst;
      t.N = axis == 0 ? mx : my;
      t.lg = 0;
      while ((1 << t.lg) < t.N) ++t.lg;
      t.tw = axis == 0 ? m->d_fftx : m->d_ffty;
      t.ph = t.tw + t.N;
      t.nl = axis == 0 ? my : mx;
      t.nslices = T * nk;
      t.sstride = (long)mx * my;
      t.lstride = axis == 0 ? mx : 1;
      t.estride = axis == 0 ? 1 : mx;
      t.inverse = inverse;
      t.tile_start = fft_tiles_total;
      fft_tiles_total += fft_tiles(t.N, (long)t.nl * t.nslices);
      fft_bytes += 16.0 * (double)mx * my * T * nk;
      ft.push_back(t);
      continue;
    }
    if (axis == 0) {
      gl.add(m->d_dctx, src, nullptr, dst, mx, my * T * nk, mx, mx, mx, mx, 1.0, 0.0, inverse, 0,
             mx, mx);
    } else {
      for (int sl = 0; sl < T * nk; ++sl) {
        const size_t o = (size_t)sl * mx * my;
        gl.add(src + o, m->d_dcty, nullptr, dst + o, mx, my, my, mx, my, mx, 1.0, 0.0, 0,
               inverse ? 0 : 1, mx, my);
      }
    }
  }
  pg.gemm(a, gl, true, RBMC_KF_DCT);
  if (!ft.empty()) {
    Op o;
    o.kind = 23;
    o.off = a.push(ft);
    o.n = (int)ft.size();
    o.tiles = fft_tiles_total;
    o.kblk = axis;
    o.max_np = 0;
    for (const FftTask& t : ft) o.max_np = std::max(o.max_np, t.N);
    o.family = RBMC_KF_DCT;
    o.alg_bytes = fft_bytes;
    pg.ops.push_back(o);
  }
  if (direct) {
    Op o;
    o.kind = 22;
    o.cols = cols;
    o.src = in;
    o.dst = out;
    o.n = axis;
    o.kblk = inverse;
    pg.ops.push_back(o);
  }
}

// z = M^-1 r over the columns of the set, tmp a work multi-vector.
void build_spectral(const std::vector<rbmc_model*>& ms, const HostCols& h, const ColSet& cols,
                    int nk, const double* r, double* z, double* tmp, Program& pg, Arena& a) {
  spectral_axis(ms, h, cols, nk, r, tmp, 0, 0, pg, a);
  spectral_axis(ms, h, cols, nk, tmp, z, 1, 0, pg, a);
  Op o;
  o.kind = 21;
  o.cols = cols;
  o.dst = z;
  o.family = RBMC_KF_SPEC_SOLVE;
  o.alg_bytes = 16.0 * (double)h.total;
  pg.ops.push_back(o);
  spectral_axis(ms, h, cols, nk, z, tmp, 1, 1, pg, a);
  spectral_axis(ms, h, cols, nk, tmp, z, 0, 1, pg, a);
}

// the per-model device views of a column set, after a model's view changed
rbmc_status upload_dms(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, hipStream_t s) {
  std::vector<DevModel> dms;
  for (rbmc_model* m : ms) dms.push_back(m->dm);
  if (!dms.empty())
    HIPCHK(hipMemcpyAsync(cx->d_dms, dms.data(), dms.size() * sizeof(DevModel),
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBMC_OK;
}

// Factor the block-Jacobi chains of every model that needs it (one program).
rbmc_status factor_bj(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, rbmc_report* rep,
                      hipStream_t s) {
  g_tune = cx->tune;
  ChainSet cs;
  for (rbmc_model* m : ms)
    if (!m->bj_ready) cs.append(m->bj);
  if (cs.size() == 0) return RBMC_OK;
  rbmc_status st = zero_info(cs, s);
  if (st != RBMC_OK) return st;
  cx->arenaA.clear();
  Program pg;
  build_twosided(cs, pg, cx->arenaA, true);
  HIPCHK(cx->arenaA.upload(s));
  st = run(cx, pg, s, cx->arenaA);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  st = check_info(cs, rep, "block-Jacobi", s);
  if (st != RBMC_OK) return st;
  for (rbmc_model* m : ms) m->bj_ready = true;
  return RBMC_OK;
}

// Block-Jacobi PCG on Q x = F z for every column of the set (caller's stream).
// z, x: multi-vectors in the column layout h (z with n + n_obs per column).
// Learned correction y = N_w(r, u) for the columns of one model, inputs
// divided by sqrt(rr[c]) and the output multiplied back (defined below).
rbmc_status learned_apply(rbmc_ctx* cx, rbmc_model* m, const double* r, const double* u,
                          const double* rr, const uint8_t* active, double* y, int ncols,
                          hipStream_t s);
bool learned_usable(const rbmc_model* m);

// Per-iteration observer of the sampler (pair generation for training): called
// after the preconditioner of iteration it, with x = x_it, r = r_it, z = M^-1 r_it.
using SampleHook = std::function<rbmc_status(int it, const double* x, const double* r,
                                             const double* z, const double* rr)>;

// b_given (single model, n x n_k): solve Q x = b instead of sampling (z unused)
rbmc_status sample_set(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, const HostCols& h,
                       const rbmc_est_opts* o, const double* z, double* x, rbmc_report* rep,
                       hipStream_t s, const SampleHook& hook = {},
                       const double* b_given = nullptr) {
  g_tune = cx->tune;
  const int nk = o->n_samples;
  double t0 = now_s();
  // the learned correction makes the preconditioner nonlinear: flexible
  // (Polak-Ribiere) PCG, z_prev kept in zp
  bool learned = false;
  if (o->precond == RBMC_PC_BJ_LEARNED)
    for (rbmc_model* m : ms) learned = learned || learned_usable(m);
  const bool spectral = o->precond == RBMC_PC_SPECTRAL;
  rbmc_status st = RBMC_OK;
  if (spectral) {
    for (rbmc_model* m : ms) {
      st = ensure_spectral(m, s);
      if (st != RBMC_OK) return st;
    }
    st = upload_dms(cx, ms, s);
  } else {
    for (rbmc_model* m : ms) {
      st = ensure_chains(m, true, nk);
      if (st != RBMC_OK) return st;
    }
    st = factor_bj(cx, ms, rep, s);
  }
  if (st != RBMC_OK) return st;
  const ColSet cols = colset(cx, h);
  const int nc = cols.ncols;
  double* r = cx->r;
  double* p = cx->p;
  double* q = cx->q;
  double* zz = cx->z;
  double* bb = cx->scal;
  double* rz = cx->scal + nc;
  double* rzn = cx->scal + 2 * nc;
  double* pq = cx->scal + 3 * nc;
  double* rr = cx->scal + 4 * nc;
  const int nch = dot_chunks(std::max(h.max_len, 1)), nsp = h.max_tiles;
  // preconditioner program: gather r -> panels, solve, scatter -> z (block
  // Jacobi), or the spectral transforms and solves
  ChainSet cs;
  if (!spectral)
    for (size_t j = 0; j < ms.size(); ++j) cs.append(ms[j]->bj);
  Arena& ar = cx->arenaA;
  ar.clear();
  Program pre, gat, sca;
  TileList<PanelTask> g, sc;
  if (spectral) {
    build_spectral(ms, h, cols, nk, r, zz, cx->zp, pre, ar);
  } else {
    size_t c0 = 0;
    for (size_t j = 0; j < ms.size(); ++j) {
      rbmc_model* m = ms[j];
      for (size_t c = 0; c < m->bj.size(); ++c) {
        const size_t cc = c0 + c;
        const Chain& ch = cs.chains[cc];
        const int np = cs.np[cc], nb = cs.nb[cc];
        for (int t = 0; t < ch.T; ++t) {
          PanelTask pt{};
          pt.P = cs.pan[cc][t];
          pt.rg = cs.rg[cc];
          pt.dm = m->d_dm;
          pt.X = r + h.base[j];
          pt.n_k = nk;
          pt.t = ch.t0 + t;
          pt.mode = 0;
          g.add(pt, panel_tiles(np, nk), 16.0 * nb * nk);
          PanelTask ps = pt;
          ps.P = cs.pan[cc][t];
          ps.X = nullptr;
          ps.Xout = zz + h.base[j];
          ps.mode = 1;
          sc.add(ps, panel_tiles(np, nk), 16.0 * nb * nk);
        }
      }
      c0 += m->bj.size();
    }
  }
  if (!spectral) {
    gat.panels(ar, g);
    // FP64 even under RBMC_MIXED: FP32-rounded solves cost the one-iteration
    // exact chain preconditioner two more iterations
    build_twisted_solve(cs, nk, pre, ar, 0, true);
    sca.panels(ar, sc);
  }
  HIPCHK(ar.upload(s));
  if (learned && cx->lws_len < h.total) {
    cx->lws.release();
    cx->lws_len = 0;
    HIPCHK(cx->lws.alloc((void**)&cx->lv, h.total * 8));
    HIPCHK(cx->lws.alloc((void**)&cx->lqv, h.total * 8));
    cx->lws_len = h.total;
  }
  if (learned)  // columns of models without a usable correction keep v = 0
    HIPCHK(hipMemsetAsync(cx->lv, 0, h.total * 8, s));
  double* vr = cx->scal + 6 * nc;
  double* vqu = cx->scal + 7 * nc;
  double* vqv = cx->scal + 8 * nc;
  // z = u + g v with u = M^-1 r, v = N_w(r, u) and the per-column step g
  // minimizing ||z - Q^-1 r||_Q (models with a usable correction);
  // rrv: the current squared residual norms.  q is free here and holds Q u.
  auto precond = [&](const double* rrv) -> rbmc_status {
    rbmc_status e = run(cx, gat, s, ar);
    if (e != RBMC_OK) return e;
    e = run(cx, pre, s, ar);
    if (e != RBMC_OK) return e;
    e = run(cx, sca, s, ar);
    if (e != RBMC_OK || !learned) return e;
    int col0 = 0;
    for (size_t j = 0; j < ms.size(); ++j) {
      if (learned_usable(ms[j])) {
        e = learned_apply(cx, ms[j], r + h.base[j], zz + h.base[j], rrv + col0,
                          cx->active + col0, cx->lv + h.base[j], nk, s);
        if (e != RBMC_OK) return e;
      }
      col0 += nk;
    }
    launch_apply_op(cols, RBMC_OP_Q, zz, q, s);
    launch_apply_op(cols, RBMC_OP_Q, cx->lv, cx->lqv, s);
    launch_dot_partials(cols, cx->lv, r, cx->part, s);
    launch_reduce_partials(cx->part, nch, nc, vr, s);
    launch_dot_partials(cols, cx->lv, q, cx->part, s);
    launch_reduce_partials(cx->part, nch, nc, vqu, s);
    launch_dot_partials(cols, cx->lv, cx->lqv, cx->part, s);
    launch_reduce_partials(cx->part, nch, nc, vqv, s);
    col0 = 0;
    for (size_t j = 0; j < ms.size(); ++j) {
      if (learned_usable(ms[j]))
        launch_gamma_axpy(cx->lv + h.base[j], zz + h.base[j], (size_t)ms[j]->plan.n, vr + col0,
                          vqu + col0, vqv + col0, cx->active + col0, nk, s);
      col0 += nk;
    }
    HIPCHK(hipGetLastError());
    return RBMC_OK;
  };
  double* rzp = cx->scal + 5 * nc;
  // b = F z (or the given b) -> r; x = 0
  if (b_given)
    HIPCHK(hipMemcpyAsync(r, b_given, h.total * 8, hipMemcpyDeviceToDevice, s));
  else
    launch_apply_op(cols, RBMC_OP_F, z, r, s);
  HIPCHK(hipMemsetAsync(x, 0, h.total * 8, s));
  launch_dot_partials(cols, r, r, cx->part, s);
  launch_reduce_partials(cx->part, nch, nc, bb, s);
  std::vector<double> hbb(nc);
  HIPCHK(hipMemcpyAsync(hbb.data(), bb, (size_t)nc * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint8_t> act(nc);
  for (int k = 0; k < nc; ++k) act[k] = hbb[k] > 0.0;
  HIPCHK(hipMemcpyAsync(cx->active, act.data(), nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(cx->iters, 0, (size_t)(nc + 1) * 4, s));
  st = precond(bb);
  if (st != RBMC_OK) return st;
  if (hook) {
    st = hook(0, x, r, zz, bb);
    if (st != RBMC_OK) return st;
  }
  launch_dot_partials(cols, r, zz, cx->part, s);
  launch_reduce_partials(cx->part, nch, nc, rz, s);
  launch_pcg_p(cols, zz, p, rz, rz, cx->active, 1, s);
  int n_active = 0;
  for (int k = 0; k < nc; ++k) n_active += act[k];
  int it = 0;
  while (n_active > 0 && it < o->pcg_maxit) {
    const int pid = cx->begin(RBMC_KF_SPMM, 0.0, 16.0 * (double)h.total, s);
    launch_spmm_dot(cols, p, q, cx->part, s);
    cx->end(pid, s);
    launch_reduce_partials(cx->part, nsp, nc, pq, s);
    launch_pcg_xr(cols, p, q, x, r, rz, pq, cx->active, cx->part, s);
    launch_reduce_partials(cx->part, nch, nc, rr, s);
    launch_pcg_check(rr, bb, o->pcg_rtol, cx->active, cx->iters + 1, cx->iters, nc, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&n_active, cx->iters, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ++it;
    if (n_active == 0) break;
    if (learned) HIPCHK(hipMemcpyAsync(cx->zp, zz, h.total * 8, hipMemcpyDeviceToDevice, s));
    st = precond(rr);
    if (st != RBMC_OK) return st;
    if (hook) {
      st = hook(it, x, r, zz, rr);
      if (st != RBMC_OK) return st;
    }
    launch_dot_partials(cols, r, zz, cx->part, s);
    launch_reduce_partials(cx->part, nch, nc, rzn, s);
    if (learned) {
      launch_dot_partials(cols, r, cx->zp, cx->part, s);
      launch_reduce_partials(cx->part, nch, nc, rzp, s);
    }
    launch_pcg_p(cols, zz, p, rzn, rz, cx->active, 0, s, learned ? rzp : nullptr);
  }
  HIPCHK(hipGetLastError());
  std::vector<int> iters(nc + 1);
  std::vector<double> hrr(nc);
  HIPCHK(hipMemcpyAsync(iters.data(), cx->iters, (size_t)(nc + 1) * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hrr.data(), rr, (size_t)nc * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (rep) {
    int itmax = 0;
    double itsum = 0.0, maxres = 0.0;
    for (int k = 0; k < nc; ++k) {
      itmax = std::max(itmax, iters[k + 1]);
      itsum += iters[k + 1];
      if (hbb[k] > 0.0) maxres = std::max(maxres, std::sqrt(hrr[k] / hbb[k]));
    }
    rep->pcg_it_max = itmax;
    rep->pcg_it_mean = nc ? itsum / nc : 0.0;
    rep->max_rel_residual = maxres;
    rep->t_sample = now_s() - t0;
  }
  return n_active > 0 ? RBMC_W_NOT_CONVERGED : RBMC_OK;
}

// Library streams of the overlapped estimate (created once per context).
// The factorization stream excludes `reserve_cus` compute units, spread
// evenly over the device, so that the sampler's chain of small serial
// kernels always finds a free CU; the other two use every CU.
rbmc_status ensure_streams(rbmc_ctx* cx) {
  if (cx->work) return RBMC_OK;
  HIPCHK(hipStreamCreateWithFlags(&cx->work, hipStreamNonBlocking));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, cx->device));
  const int ncu = prop.multiProcessorCount;
  const int r = cx->reserve_cus;
  if (r > 0 && r < ncu) {
    const int stride = ncu / r;
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int i = 0; i < ncu; ++i)
      if (i % stride != stride - 1 || i / stride >= r) mask[i / 32] |= 1u << (i % 32);
    for (hipStream_t* st : {&cx->side, &cx->side2})
      if (hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        *st = nullptr;
      } else {
        cx->cu_masked = true;
      }
  }
  if (!cx->side) HIPCHK(hipStreamCreateWithFlags(&cx->side, hipStreamNonBlocking));
  if (!cx->side2) HIPCHK(hipStreamCreateWithFlags(&cx->side2, hipStreamNonBlocking));
  for (hipEvent_t& e : cx->join) HIPCHK(hipEventCreate(&e));
  return RBMC_OK;
}

// Partial-sum layout of the estimator over a list of subdomain chains: per
// chain and local step, the deterministic slots (diagonal block, off-diagonal
// t -> t+1, t+1 -> t) in chunks of 256 rows with 3 sums each, and the Monte
// Carlo sums in chunks of 64 rows with 8 sums each.
struct EstLayout {
  std::vector<Chain> ch;
  std::vector<const rbmc_model*> owner;
  std::vector<int> np, cmodel;
  std::vector<size_t> det_base, mc_base;
  size_t det_len = 0, mc_len = 0;
  void add(const Chain& c, const rbmc_model* m, int np_, int model) {
    ch.push_back(c);
    owner.push_back(m);
    np.push_back(np_);
    cmodel.push_back(model);
  }
  void finish() {
    const size_t n = ch.size();
    det_base.assign(n + 1, 0);
    mc_base.assign(n + 1, 0);
    for (size_t c = 0; c < n; ++c) {
      det_base[c + 1] = det_base[c] + (size_t)ch[c].T * 3 * nchk(c);
      mc_base[c + 1] = mc_base[c] + (size_t)ch[c].T * mc_chunks(np[c]);
    }
    det_len = det_base[n] * 3;
    mc_len = mc_base[n] * 8;
  }
  size_t nchk(size_t c) const { return (np[c] + 255) / 256; }
  size_t det_index(size_t c, int t, int sl) const {
    return det_base[c] + ((size_t)t * 3 + sl) * nchk(c);
  }
  size_t mc_index(size_t c, int t) const { return mc_base[c] + (size_t)t * mc_chunks(np[c]); }
};

// Device partial sums of a layout (the context's estimator buffer).
rbmc_status ensure_epart(rbmc_ctx* cx, const EstLayout& L) {
  const size_t need = std::max<size_t>(L.det_len + L.mc_len, 1);
  if (cx->epart_len < need) {
    cx->epool.release();
    cx->epart_len = 0;
    HIPCHK(cx->epool.alloc((void**)&cx->epart, need * 8));
    cx->epart_len = need;
  }
  return RBMC_OK;
}

// Alg. 2: the separator nodes' variance from the samples (x in the column
// layout h, nk columns per model, each scaled by `scale`); accum = 0 starts
// from zero.  Models without separators are skipped.
void sep_variance(const std::vector<rbmc_model*>& ms, const HostCols& h, int nk, const double* x,
                  double scale, int accum, const std::vector<double*>& diag_out, hipStream_t s) {
  for (size_t j = 0; j < ms.size(); ++j) {
    const rbmc_model* m = ms[j];
    const int nsep = (int)m->plan.sep_nodes.size();
    if (nsep == 0) continue;
    launch_sep_var(m->d_sep, nsep, x ? x + h.base[j] : nullptr, m->plan.n, x ? nk : 0, scale,
                   accum, diag_out[j], s);
  }
}

// Alg. 2 defines variances only: no traces with separators
rbmc_status sep_check(const std::vector<rbmc_model*>& ms, const rbmc_est_opts* o) {
  for (const rbmc_model* m : ms)
    if (m->plan.sep && o->grad_mask)
      return fail(RBMC_E_UNSUPPORTED, "traces are not defined with separators (Alg. 2)");
  return RBMC_OK;
}

// Traces and the plug-in error from the partial sums (host, fixed order):
// the deterministic and Monte Carlo Frobenius products of each core step
// weighted by the time coefficients of dQ_j (eq:hyperpar:4).
rbmc_status combine_traces(rbmc_ctx* cx, const EstLayout& L, const std::vector<rbmc_model*>& ms,
                           int nk, const rbmc_est_opts* o,
                           const std::vector<double*>& trace_out, rbmc_report* rep) {
  std::vector<double> hpart(L.det_len + L.mc_len);
  HIPCHK(hipMemcpy(hpart.data(), cx->epart, (L.det_len + L.mc_len) * 8, hipMemcpyDeviceToHost));
  const double* hdet = hpart.data();
  const double* hmc = hpart.data() + L.det_len;
  std::vector<std::array<double, 4>> tr(ms.size(), {0.0, 0.0, 0.0, 0.0});
  double ratio_sum = 0.0;  // sum over nodes of (MC part) / (estimate)
  size_t n_total = 0;
  for (rbmc_model* m : ms) n_total += m->plan.n;
  for (size_t c = 0; c < L.ch.size(); ++c) {
    const Chain& ch = L.ch[c];
    const Coefs& co = L.owner[c]->co;
    const size_t nchk = L.nchk(c), mchk = mc_chunks(L.np[c]);
    const int lc0 = ch.ct0 - ch.t0, lc1 = lc0 + ch.cT - 1;
    for (int t = lc0; t <= lc1; ++t) {
      const int tg = ch.t0 + t;
      // deterministic: slot 0 (t,t), slot 1 (t,t+1), slot 2 (t,t-1)
      double Fd = 0, Fq[3] = {0, 0, 0}, Fk[3] = {0, 0, 0};
      for (int sl = 0; sl < 3; ++sl)
        for (size_t k = 0; k < nchk; ++k) {
          const double* pp = &hdet[(L.det_index(c, t, sl) + k) * 3];
          if (sl == 0) Fd += pp[0];
          Fq[sl] += pp[1];
          Fk[sl] += pp[2];
        }
      // Monte Carlo: components [t-1, t, t+1] for Q_s and K, then D, then m/s2
      double G[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (nk > 0)
        for (size_t k = 0; k < mchk; ++k)
          for (int j = 0; j < 8; ++j) G[j] += hmc[(L.mc_index(c, t) + k) * 8 + j];
      ratio_sum += G[7];
      const double wq0 = co.qd[tg], wqo = co.qo, wd0 = co.dqd[tg], wdo = co.dqo;
      const bool hm = (t - 1 >= 0), hp = (t + 1 < ch.T);
      const double q_tt = Fq[0] + G[1];
      const double q_tp = hp ? Fq[1] + G[2] : 0.0;
      const double q_tm = hm ? Fq[2] + G[0] : 0.0;
      const double k_tt = Fk[0] + G[4];
      const double k_tp = hp ? Fk[1] + G[5] : 0.0;
      const double k_tm = hm ? Fk[2] + G[3] : 0.0;
      std::array<double, 4>& T = tr[L.cmodel[c]];
      T[0] += wq0 * k_tt + wqo * (k_tp + k_tm);
      T[1] += wq0 * q_tt + wqo * (q_tp + q_tm);
      T[2] += wd0 * q_tt + wdo * (q_tp + q_tm);
      T[3] += -2.0 * (Fd + G[6]);
    }
  }
  for (size_t j = 0; j < ms.size(); ++j)
    if (trace_out[j]) {
      int k = 0;
      for (int b = 0; b < 4; ++b)
        if (o->grad_mask & (1u << b)) trace_out[j][k++] = tr[j][b];
    }
  // Alg. 2 separator nodes: their estimate is all Monte Carlo (ratio 1)
  if (nk > 0)
    for (const rbmc_model* m : ms) ratio_sum += (double)m->plan.sep_nodes.size();
  if (rep) {
    // plug-in MC error: m_i ~ E[mu_i^2] chi2_{n_k} / n_k, so the mean absolute relative
    // error of the estimate is about sqrt(2/pi) sqrt(2/n_k) m_i / s2_i on average
    rep->err_estimate =
        nk > 0 ? std::sqrt(2.0 / M_PI) * std::sqrt(2.0 / nk) * ratio_sum / (double)n_total : 0.0;
  }
  return RBMC_OK;
}

// The estimator from samples for a set of models.  x_base: the samples in the
// column layout h (ignored when n_k = 0).  The subdomain factorization and the
// core steps do not need the samples: when `sampler` is given they run on
// the side stream while sampler() produces x on the caller's stream, and the
// two streams join before the correction solves.
rbmc_status estimate_set(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, const HostCols& h,
                         const rbmc_est_opts* o, const double* x_base,
                         const std::vector<double*>& diag_out,
                         const std::vector<double*>& trace_out, rbmc_report* rep,
                         const std::function<rbmc_status()>& sampler) {
  g_tune = cx->tune;
  const int nk = o->n_samples;
  const int mixed = o->precision == RBMC_MIXED;
  {
    rbmc_status e = sep_check(ms, o);
    if (e != RBMC_OK) return e;
  }
  if (sampler) {
    rbmc_status e = ensure_streams(cx);
    if (e != RBMC_OK) return e;
  }
  // sA: sampler (when overlapped) and corrections; s: two-sided
  // factorization; sT: core steps
  hipStream_t sA = sampler ? cx->work : cx->stream;
  hipStream_t s = sampler ? cx->side : sA;
  hipStream_t sT = sampler ? cx->side2 : sA;
  double t0 = now_s();
  for (rbmc_model* m : ms) {
    rbmc_status e = ensure_chains(m, false, nk);
    if (e != RBMC_OK) return e;
  }
  EstLayout L;
  for (size_t j = 0; j < ms.size(); ++j)
    for (size_t c = 0; c < ms[j]->sub.size(); ++c)
      L.add(ms[j]->sub.chains[c], ms[j], ms[j]->sub.np[c], (int)j);
  L.finish();
  {
    rbmc_status e = ensure_epart(cx, L);
    if (e != RBMC_OK) return e;
  }
  const size_t need = std::max<size_t>(L.det_len + L.mc_len, 1);
  double* det_part = cx->epart;
  double* mc_part = cx->epart + L.det_len;
  auto det_index = [&](int c, int t, int sl) { return L.det_index(c, t, sl); };
  auto mc_index = [&](int c, int t) { return L.mc_index(c, t); };
  // combined subdomain chain set and per-chain model index
  ChainSet cs;
  std::vector<int> cmodel;
  for (size_t j = 0; j < ms.size(); ++j) {
    cs.append(ms[j]->sub);
    cmodel.insert(cmodel.end(), ms[j]->sub.size(), (int)j);
  }
  ChainSet cf;  // chains that need factoring now
  for (rbmc_model* m : ms)
    if (!m->sub_ready) cf.append(m->sub);
  const int nchains = (int)cs.size();
  Arena& ar = cx->arenaB;
  ar.clear();
  Program fac;
  if (cf.size()) build_twosided(cf, fac, ar);
  auto lc0 = [&](int c) { return cs.chains[c].ct0 - cs.chains[c].t0; };
  auto lc1 = [&](int c) { return lc0(c) + cs.chains[c].cT - 1; };
  auto is_core = [&](int c, int t) { return t >= lc0(c) && t <= lc1(c); };
  auto etask = [&](int c, const double* M, int t, int kind, int trans, double sign, int sl) {
    ExtractTask e{};
    e.M = M;
    e.ld = cs.np[c];
    e.rg = cs.rg[c];
    e.dm = cs.owner[c]->d_dm;
    e.diag_out = diag_out[cmodel[c]];
    e.partial = det_part;
    e.out_index = (int)det_index(c, t, sl);
    e.t = cs.chains[c].t0 + t;
    e.kind = kind;
    e.trans = trans;
    e.sign = sign;
    return e;
  };

  // ---- core steps: Sigma_tt = (B_t - q_o^2 Q_R (F_{t-1} + G_{t+1}) Q_R)^-1,
  // its diagonal and stencil entries, and the stencil entries of the
  // off-diagonal blocks Sigma_{t,t+1} = -q_o (G_{t+1} Q_R Sigma_tt)^T and
  // Sigma_{t,t-1} = -q_o (F_{t-1} Q_R Sigma_tt)^T.  Core step k of every
  // chain per round (sig holds the first core step for the solves).
  Program tak;
  {
    int max_ct = 0;
    for (int c = 0; c < nchains; ++c) max_ct = std::max(max_ct, cs.chains[c].cT);
    for (int k = 0; k < max_ct; ++k) {
      StencilList v1, v2, wp, wm;
      std::vector<InvJob> inv;
      TileList<ExtractTask> ex;
      TileList<OffdiagTask> op, om;
      for (int c = 0; c < nchains; ++c) {
        const Chain& ch = cs.chains[c];
        if (k >= ch.cT) continue;
        const int t = lc0(c) + k;
        const int np = cs.np[c], nb = cs.nb[c];
        const double qo = cs.owner[c]->co.qo;
        double* sg = (k == 0) ? cs.sig[c] : cs.sig2[c];
        const double* Fm = (t >= 1) ? fblock(cs, c, t - 1) : nullptr;
        const double* Gp = (t + 1 < ch.T) ? gblock(cs, c, t + 1) : nullptr;
        add_schur(cs, c, t, Fm, Gp, sg, v1, v2);
        inv.push_back(inv_job(cs, c, sg));
        ex.add(etask(c, sg, t, 0, 0, 1.0, 0), (np + 255) / 256);
        for (int side = 0; side < 2; ++side) {
          const double* far = side == 0 ? Gp : Fm;
          if (!far) continue;
          StencilTask w = stask(cs, c);  // W = Q_R (far inverse), column-major
          w.M = far;
          w.ldm = np;
          w.alpha = 1.0;
          w.out = cs.tmp[c];
          w.ldout = np;
          w.ncols = np;
          (side == 0 ? wp : wm).add(w, np, nb);
          OffdiagTask o{};
          o.W = cs.tmp[c];
          o.Sig = sg;
          o.ld = np;
          o.rg = cs.rg[c];
          o.dm = cs.owner[c]->d_dm;
          o.partial = det_part;
          o.out_index = (int)det_index(c, t, side == 0 ? 1 : 2);
          o.scale = -qo;
          (side == 0 ? op : om).add(o, (np + 255) / 256, 16.0 * nb * (double)nb);
        }
      }
      tak.stencil(ar, v1);
      tak.stencil(ar, v2);
      tak.inverse(ar, inv);
      tak.extract(ar, ex);
      tak.stencil(ar, wp);
      tak.offdiag(ar, op);
      tak.stencil(ar, wm);
      tak.offdiag(ar, om);
    }
  }
  // ---- corrections ----
  Program cor;
  if (nk > 0) {
    TileList<PanelTask> rt;
    for (int c = 0; c < nchains; ++c) {
      const Chain& ch = cs.chains[c];
      const int np = cs.np[c];
      for (int t = 0; t < ch.T; ++t) {
        PanelTask pt{};
        pt.P = cs.pan[c][t];
        pt.rg = cs.rg[c];
        pt.dm = cs.owner[c]->d_dm;
        pt.X = x_base + h.base[cmodel[c]];
        pt.n_k = nk;
        pt.t = ch.t0 + t;
        pt.t0 = ch.t0;
        pt.T = ch.T;
        pt.mode = 2;
        rt.add(pt, panel_tiles(np, nk), 16.0 * cs.nb[c] * nk);
      }
    }
    cor.panels(ar, rt);
    build_twisted_solve(cs, nk, cor, ar, mixed);
    TileList<McTask> mt;
    for (int c = 0; c < nchains; ++c) {
      const Chain& ch = cs.chains[c];
      for (int t = lc0(c); t <= lc1(c); ++t) {
        McTask k{};
        k.mu[0] = (t - 1 >= 0) ? cs.pan[c][t - 1] : nullptr;
        k.mu[1] = cs.pan[c][t];
        k.mu[2] = (t + 1 < ch.T) ? cs.pan[c][t + 1] : nullptr;
        k.np = cs.np[c];
        k.rg = cs.rg[c];
        k.dm = cs.owner[c]->d_dm;
        k.diag_out = diag_out[cmodel[c]];
        k.partial = mc_part;
        k.out_index = (int)mc_index(c, t);
        k.n_k = nk;
        k.scale = 1.0 / nk;
        k.accum = 0;
        k.t = ch.t0 + t;
        mt.add(k, mc_chunks(cs.np[c]), 8.0 * cs.nb[c] * nk);
      }
    }
    cor.mc(ar, mt);
  }
  // the library streams start after everything already queued on the caller's stream
  if (sampler) {
    HIPCHK(hipEventRecord(cx->join[0], cx->stream));
    HIPCHK(hipStreamWaitEvent(s, cx->join[0], 0));
    HIPCHK(hipStreamWaitEvent(sA, cx->join[0], 0));
  }
  HIPCHK(ar.upload(s));
  HIPCHK(hipMemsetAsync(cx->epart, 0, need * 8, s));
  {  // the core-step inversions run on every call
    rbmc_status st0 = zero_info(cs, s);
    if (st0 != RBMC_OK) return st0;
  }
  hipEvent_t e_fac = nullptr, e_tak = nullptr, e_beg = nullptr;
  if (cx->join[1]) {
    e_beg = cx->join[1];
    e_fac = cx->join[2];
    e_tak = cx->join[3];
    HIPCHK(hipEventRecord(e_beg, s));
  }
  // factorization on stream s and the core steps on sT; with a sampler they are enqueued
  // by a second host thread, so neither stream waits for the host to finish
  // enqueuing the other's launches (a stream's queue fills up long before
  // thousands of launches are placed, and placing then blocks).
  rbmc_status st_b = RBMC_OK;
  std::string err_b;
  auto side_work = [&]() {
    if (sampler && hipSetDevice(cx->device) != hipSuccess) {
      st_b = fail(RBMC_E_DEVICE, "hipSetDevice failed on the launch thread");
    }
    if (st_b == RBMC_OK) st_b = run(cx, fac, s, ar);
    if (st_b == RBMC_OK && e_fac && hipEventRecord(e_fac, s) != hipSuccess)
      st_b = fail(RBMC_E_DEVICE, "hipEventRecord failed");
    if (st_b == RBMC_OK && sT != s && hipStreamWaitEvent(sT, e_fac, 0) != hipSuccess)
      st_b = fail(RBMC_E_DEVICE, "hipStreamWaitEvent failed");
    if (st_b == RBMC_OK) st_b = run(cx, tak, sT, ar);
    if (st_b == RBMC_OK && e_tak && hipEventRecord(e_tak, sT) != hipSuccess)
      st_b = fail(RBMC_E_DEVICE, "hipEventRecord failed");
    if (st_b != RBMC_OK) err_b = g_err;
  };
  rbmc_status st_samp = RBMC_OK;
  if (sampler) {
    if (cx->launch_threads) {
      std::thread tb(side_work);
      st_samp = sampler();  // on the caller's stream, concurrently with the side stream
      tb.join();
    } else {
      side_work();
      st_samp = sampler();
    }
    if (st_b != RBMC_OK) {
      (void)hipStreamSynchronize(sA);
      (void)hipStreamSynchronize(s);
      (void)hipStreamSynchronize(sT);
      return fail(st_b, err_b);
    }
    if (st_samp < 0) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamSynchronize(sT);
      return st_samp;
    }
    HIPCHK(hipStreamWaitEvent(sA, e_tak, 0));
  } else {
    side_work();
    if (st_b != RBMC_OK) return st_b;
  }
  rbmc_status st = RBMC_OK;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipStreamSynchronize(sT));
  st = check_info(cs, rep, "subdomain", sA);
  if (st != RBMC_OK) return st;
  for (rbmc_model* m : ms) m->sub_ready = true;
  double t2 = now_s();
  st = run(cx, cor, sA, ar);
  if (st != RBMC_OK) return st;
  if (sA != cx->stream) {
    HIPCHK(hipEventRecord(cx->join[4], sA));
    HIPCHK(hipStreamWaitEvent(cx->stream, cx->join[4], 0));
  }
  HIPCHK(hipStreamSynchronize(sA));
  double t3 = now_s();
  float ms_fac = 0.f, ms_tak = 0.f;
  if (e_beg) {
    HIPCHK(hipEventElapsedTime(&ms_fac, e_beg, e_fac));
    HIPCHK(hipEventElapsedTime(&ms_tak, e_fac, e_tak));
  }
  sep_variance(ms, h, nk, x_base, nk > 0 ? 1.0 / nk : 0.0, 0, diag_out, cx->stream);
  HIPCHK(hipGetLastError());
  // ---- traces: combine partial sums with the temporal weights ----
  st = combine_traces(cx, L, ms, nk, o, trace_out, rep);
  if (st != RBMC_OK) return st;
  if (rep) {
    rep->t_factor = ms_fac * 1e-3;
    rep->t_select = ms_tak * 1e-3;
    rep->t_correct = t3 - t2;
    int64_t bytes = cx->ws.bytes + cx->epool.bytes;
    for (rbmc_model* m : ms)
      bytes += m->pool.bytes + m->work_bj.bytes + m->work_sub.bytes + m->kpool.bytes +
               m->spool.bytes;
    rep->peak_bytes = bytes;
  }
  (void)t0;
  return st_samp;
}


// ---------------------------------------------------------------------------
// Learned correction N_w: 4 convolutions 3^3 (2 -> 16 -> 16 -> 16 -> 1), ReLU
// between them, no bias (so N_w(a r, a u) = a N_w(r, u) for a > 0), on the
// space-time grid of each sample; inputs r and u = M_BJ^-1 r.  Weights:
// layer l occupies [kWOff[l], kWOff[l+1]).
// ---------------------------------------------------------------------------
constexpr int kNL = 4;
constexpr int kCin[kNL] = {2, 16, 16, 16};
constexpr int kCout[kNL] = {16, 16, 16, 1};
constexpr int kWOff[kNL + 1] = {0, 864, 864 + 6912, 864 + 2 * 6912, 864 + 2 * 6912 + 432};
constexpr int kNW = kWOff[kNL];
static_assert(kNW == RBMC_PC_NWEIGHTS, "weight count");

bool learned_usable(const rbmc_model* m) { return m->lrn.ready && m->lrn.usable; }

rbmc_status ensure_learned(rbmc_model* m) {
  if (m->lrn.w) return RBMC_OK;
  HIPCHK(m->pool.alloc((void**)&m->lrn.w, kNW * 4));
  HIPCHK(m->pool.alloc((void**)&m->lrn.wb, kNW * 2));
  HIPCHK(m->pool.alloc((void**)&m->lrn.wf, kNW * 2));
  HIPCHK(m->pool.alloc((void**)&m->lrn.am, kNW * 4));
  HIPCHK(m->pool.alloc((void**)&m->lrn.av, kNW * 4));
  HIPCHK(m->pool.alloc((void**)&m->lrn.g, kNW * 4));
  return RBMC_OK;
}

// BF16 copy and flipped/transposed copy of the FP32 weights
void learned_derive(rbmc_model* m, hipStream_t s) {
  launch_to_bf16(m->lrn.w, m->lrn.wb, kNW, s);
  for (int l = 0; l < kNL; ++l)
    launch_conv_wflip(m->lrn.wb + kWOff[l], kCin[l], kCout[l], m->lrn.wf + kWOff[l], s);
}

ConvGeom model_geom(const rbmc_model* m) { return ConvGeom{m->plan.T, m->plan.my, m->plan.mx}; }

// Forward pass over `batch` volumes: in (B x 2 x V) -> out (B x 1 x V);
// h[0..2]: B x 16 x V pre-activations (h[2] may alias h[0]).
void learned_forward(const rbmc_model* m, ConvGeom g, int batch, const float* in,
                     float* const h[3], float* out, hipStream_t s) {
  const float* src = in;
  for (int l = 0; l < kNL; ++l) {
    ConvArgs a{};
    a.in = src;
    a.out = (l == kNL - 1) ? out : h[l];
    a.w = m->lrn.wb + kWOff[l];
    a.geom = g;
    a.relu_in = l > 0;
    a.scale = 1.f;
    launch_conv3d(a, kCin[l], kCout[l], batch, s);
    src = a.out;
  }
}

rbmc_status learned_apply(rbmc_ctx* cx, rbmc_model* m, const double* r, const double* u,
                          const double* rr, const uint8_t* active, double* y, int ncols,
                          hipStream_t s) {
  (void)cx;
  const ConvGeom g = model_geom(m);
  const size_t V = (size_t)m->plan.n;
  // columns per chunk: input (2 channels), output, two 16-channel buffers, within ~4 GB
  const size_t per_col = V * 4 * (2 + 1 + 16 + 16);
  const int cb = (int)std::max<size_t>(1, std::min<size_t>(ncols, ((size_t)4 << 30) / per_col));
  if (m->lwork_cols < (size_t)cb) {
    m->lwork.release();
    m->lwork_cols = 0;
    float* p = nullptr;
    HIPCHK(m->lwork.alloc((void**)&p, per_col * cb));
    m->lwork_cols = cb;
  }
  float* base = (float*)m->lwork.ptrs[0];
  float* vin = base;
  float* vout = vin + 2 * V * cb;
  float* ha = vout + V * cb;
  float* hb = ha + 16 * V * cb;
  float* const hs[3] = {ha, hb, ha};
  for (int c0 = 0; c0 < ncols; c0 += cb) {
    const int nc = std::min(cb, ncols - c0);
    launch_cols2_to_vol(r + (size_t)c0 * V, u + (size_t)c0 * V, V, rr ? rr + c0 : nullptr, vin,
                        nc, s);
    learned_forward(m, g, nc, vin, hs, vout, s);
    launch_vol_to_cols(vout, V, rr ? rr + c0 : nullptr, active ? active + c0 : nullptr,
                       y + (size_t)c0 * V, nc, 0, s);
  }
  HIPCHK(hipGetLastError());
  return RBMC_OK;
}

// Scale the first layer's u-channel weights by a and the last layer by b
// (host round trip; used to fold / unfold the input and output scales).
rbmc_status learned_rescale(rbmc_model* m, double a, double b, hipStream_t s) {
  std::vector<float> w(kNW);
  HIPCHK(hipMemcpyAsync(w.data(), m->lrn.w, kNW * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int co = 0; co < kCout[0]; ++co)
    for (int k = 0; k < 27; ++k) w[(co * kCin[0] + 1) * 27 + k] = (float)(w[(co * kCin[0] + 1) * 27 + k] * a);
  for (int i = kWOff[kNL - 1]; i < kWOff[kNL]; ++i) w[i] = (float)(w[i] * b);
  HIPCHK(hipMemcpyAsync(m->lrn.w, w.data(), kNW * 4, hipMemcpyHostToDevice, s));
  learned_derive(m, s);
  HIPCHK(hipStreamSynchronize(s));
  return RBMC_OK;
}

// Training of N_w on pairs generated by the sampler itself.  A first
// block-Jacobi PCG run on the given right-hand sides, 1000 times tighter than
// the caller's tolerance, gives x*; an identical second run stops at n_sel
// evenly spaced iterations k in the first three quarters of its iterations
// (so that x* - x_k is accurate to about 1e-3); every column there gives a
// pair (r_k, u_k, e_k) / |r_k| with u_k = M^-1 r_k and e_k = x* - x_k
// (Q e_k = r_k).  The network sees (r, s u) and its output y gives the
// correction y / s, with s the RMS ratio of r to u over the pairs (folded into
// the weights afterwards).  Adam minimizes the mean over a batch of the
// relative energy error ||u + y / s - e||_Q^2 / (e . r) on whole grids; the
// last tenth of the pairs is held out.
rbmc_status precond_train(rbmc_model* m, const rbmc_est_opts* po, const rbmc_train_opts* to,
                          const double* z, int n_train, float* loss_out, rbmc_report* rep) {
  rbmc_ctx* cx = m->ctx;
  hipStream_t s = cx->stream;
  rbmc_status st = ensure_learned(m);
  if (st != RBMC_OK) return st;
  const ConvGeom g = model_geom(m);
  const size_t n = (size_t)m->plan.n;
  const int npairs = std::max(to->n_pairs, 2);
  if ((double)npairs * n * 12.0 > 16.0 * (1ull << 30))
    return fail(RBMC_E_ARG, "training pairs exceed 16 GiB (reduce n_pairs)");
  std::mt19937_64 rng(to->seed);
  const bool fresh = !m->lrn.ready;
  if (fresh) {
    // He-scaled normals; the last layer zero, so training starts from block Jacobi
    std::vector<float> w(kNW, 0.f);
    for (int l = 0; l < kNL - 1; ++l) {
      std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (kCin[l] * 27.f)));
      for (int i = kWOff[l]; i < kWOff[l + 1]; ++i) w[i] = nd(rng);
    }
    HIPCHK(hipMemcpyAsync(m->lrn.w, w.data(), kNW * 4, hipMemcpyHostToDevice, s));
    learned_derive(m, s);
  }
  HIPCHK(hipMemsetAsync(m->lrn.am, 0, kNW * 4, s));
  HIPCHK(hipMemsetAsync(m->lrn.av, 0, kNW * 4, s));
  // ---- pairs from the sampler ----
  rbmc_est_opts o = *po;
  o.n_samples = n_train;
  o.precond = RBMC_PC_BJ;
  o.pcg_rtol = std::max(std::min(po->pcg_rtol, 1e-8) * 1e-3, 1e-14);
  o.pcg_maxit = std::max(po->pcg_maxit, 1) * 2;
  std::vector<rbmc_model*> ms{m};
  const HostCols h = make_cols(ms, n_train);
  st = ensure_ws(cx, ms, h, false);
  if (st != RBMC_OK) return st;
  st = ensure_chains(m, true, n_train);
  if (st != RBMC_OK) return st;
  Pool tp;  // training data, released on return
  struct Release {
    Pool& p;
    ~Release() { p.release(); }
  } rel{tp};
  double* xs = nullptr;
  float *R = nullptr, *U = nullptr, *E = nullptr;
  int* dslot = nullptr;
  HIPCHK(tp.alloc((void**)&xs, n * n_train * 8));
  HIPCHK(tp.alloc((void**)&R, n * npairs * 4));
  HIPCHK(tp.alloc((void**)&U, n * npairs * 4));
  HIPCHK(tp.alloc((void**)&E, n * npairs * 4));
  HIPCHK(tp.alloc((void**)&dslot, (size_t)std::max(n_train, npairs) * 4));
  rbmc_report r1{};
  st = sample_set(cx, ms, h, &o, z, xs, &r1, s);
  if (st < 0) return st;
  const int nit = std::max(r1.pcg_it_max, 1);
  const int span = std::max(1, (3 * nit) / 4);
  const int n_sel = std::max(1, std::min(span, (npairs + n_train - 1) / n_train));
  std::vector<int> sel_it(n_sel);
  for (int i = 0; i < n_sel; ++i) sel_it[i] = (int)((long long)i * span / n_sel);
  int made = 0, next_sel = 0;
  std::vector<double> hrr(n_train);
  std::vector<int> cslot(n_train), pair_col;
  // the last quarter of the columns is held out: its pairs validate, and the
  // acceptance trial runs on its right-hand sides
  const int n_hold = std::max(1, n_train / 4);
  const int c_hold = n_train - n_hold;
  SampleHook hook = [&](int it, const double* x, const double* r, const double* zk,
                        const double* rrv) -> rbmc_status {
    if (next_sel >= n_sel || made >= npairs) return RBMC_W_NOT_CONVERGED;  // done: stop the run
    if (it != sel_it[next_sel]) return RBMC_OK;
    ++next_sel;
    HIPCHK(hipMemcpyAsync(hrr.data(), rrv, n_train * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < n_train; ++c) {
      cslot[c] = (hrr[c] > 0.0 && made < npairs) ? made++ : -1;
      if (cslot[c] >= 0) pair_col.push_back(c);
    }
    HIPCHK(hipMemcpyAsync(dslot, cslot.data(), n_train * 4, hipMemcpyHostToDevice, s));
    launch_pair_store(r, zk, xs, x, n, rrv, dslot, R, U, E, n_train, s);
    HIPCHK(hipStreamSynchronize(s));  // dslot is reused by the next stop
    return RBMC_OK;
  };
  rbmc_report r2{};
  st = sample_set(cx, ms, h, &o, z, cx->x, &r2, s, hook);
  if (st < 0) return st;
  if (made < 2) return fail(RBMC_E_ARG, "too few training pairs (the sampler converged at once)");
  const int np_used = made;
  // per-pair e . r (= ||e||_Q^2) and the input scale s = RMS(r) / RMS(u)
  const int nblk = 64;
  double* part = nullptr;
  HIPCHK(tp.alloc((void**)&part, (size_t)std::max(np_used, 8) * nblk * 8));
  {
    std::vector<int> iota(np_used);
    for (int i = 0; i < np_used; ++i) iota[i] = i;
    HIPCHK(hipMemcpyAsync(dslot, iota.data(), np_used * 4, hipMemcpyHostToDevice, s));
  }
  auto pair_sums = [&](const float* a, const float* b2, std::vector<double>& out) -> rbmc_status {
    launch_energy_dot(nullptr, a, dslot, nullptr, b2, n, nullptr, nullptr, part, nblk, np_used, s);
    std::vector<double> hp((size_t)np_used * nblk);
    HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.assign(np_used, 0.0);
    for (int i = 0; i < np_used; ++i)
      for (int k = 0; k < nblk; ++k) out[i] += hp[(size_t)i * nblk + k];
    return RBMC_OK;
  };
  std::vector<double> eref, rsq, usq;
  if ((st = pair_sums(E, R, eref)) != RBMC_OK) return st;
  if ((st = pair_sums(R, R, rsq)) != RBMC_OK) return st;
  if ((st = pair_sums(U, U, usq)) != RBMC_OK) return st;
  double sr = 0.0, su2 = 0.0;
  for (int i = 0; i < np_used; ++i) {
    sr += rsq[i];
    su2 += usq[i];
  }
  const double su = (sr > 0.0 && su2 > 0.0) ? std::sqrt(sr / su2) : 1.0;
  // pairs with a positive energy (all, in exact arithmetic): fitted ones from
  // the training columns, held-out ones from the last n_hold columns
  std::vector<int> fit, val;
  for (int i = 0; i < np_used; ++i)
    if (eref[i] > 0.0) (pair_col[i] < c_hold ? fit : val).push_back(i);
  if (fit.empty() || val.empty())
    return fail(RBMC_E_ARG, "too few training pairs (need n_train >= 2 and unconverged columns)");
  std::vector<int> order(fit);
  order.insert(order.end(), val.begin(), val.end());
  if (!fresh) {  // continue from folded weights: unfold for the scaled inputs
    st = learned_rescale(m, 1.0 / su, su, s);
    if (st != RBMC_OK) return st;
  }
  // ---- training ----
  const int B = std::max(1, std::min(to->batch > 0 ? to->batch : 8, (int)fit.size()));
  const int n_val = (int)val.size();
  const int n_fit = (int)fit.size();
  const HostCols hB = make_cols(ms, B);
  st = ensure_ws(cx, ms, hB, false);
  if (st != RBMC_OK) return st;
  const ColSet cB = colset(cx, hB);
  float *bin = nullptr, *hbuf = nullptr, *gbuf = nullptr, *yout = nullptr, *gy = nullptr,
        *wpart = nullptr, *dcoef = nullptr;
  double *dcol = nullptr, *qd = nullptr;
  int* bslot = nullptr;
  HIPCHK(tp.alloc((void**)&bin, n * B * 2 * 4));
  HIPCHK(tp.alloc((void**)&hbuf, n * B * 16 * 3 * 4));
  HIPCHK(tp.alloc((void**)&gbuf, n * B * 16 * 2 * 4));
  HIPCHK(tp.alloc((void**)&yout, n * B * 4));
  HIPCHK(tp.alloc((void**)&gy, n * B * 4));
  HIPCHK(tp.alloc((void**)&dcol, n * B * 8));
  HIPCHK(tp.alloc((void**)&qd, n * B * 8));
  HIPCHK(tp.alloc((void**)&bslot, (size_t)B * 4));
  HIPCHK(tp.alloc((void**)&dcoef, (size_t)B * 4));
  const int wt_tiles = conv_wgrad_tiles(g);
  HIPCHK(tp.alloc((void**)&wpart, (size_t)wt_tiles * B * 16 * 16 * 27 * 4));
  float* const hs[3] = {hbuf, hbuf + n * B * 16, hbuf + n * B * 32};
  float* ga = gbuf;
  float* gb = gbuf + n * B * 16;
  std::vector<int> hsl(B);
  std::vector<float> hcoef(B);
  std::vector<double> hp((size_t)B * nblk);
  // energy error of a batch (per pair: d^T Q d / (e . r)); with_net false:
  // block Jacobi alone; grad: also the output gradient in gy
  auto batch_energy = [&](const std::vector<int>& ids, int i0, int nb, bool with_net, bool grad,
                          std::vector<double>& out) -> rbmc_status {
    for (int k = 0; k < nb; ++k) {
      hsl[k] = ids[i0 + k];
      hcoef[k] = (float)(2.0 / (su * eref[hsl[k]] * nb));
    }
    HIPCHK(hipMemcpyAsync(bslot, hsl.data(), nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dcoef, hcoef.data(), nb * 4, hipMemcpyHostToDevice, s));
    if (with_net) {
      launch_pack_train(R, U, bslot, n, (float)su, bin, nb, s);
      learned_forward(m, g, nb, bin, hs, yout, s);
    }
    launch_energy_d(U, E, with_net ? yout : nullptr, bslot, n, (float)(1.0 / su), dcol, nb, s);
    ColSet c = cB;
    c.ncols = nb;
    launch_apply_op(c, RBMC_OP_Q, dcol, qd, s);
    launch_energy_dot(dcol, nullptr, bslot, qd, nullptr, n, dcoef, grad ? gy : nullptr, part,
                      nblk, nb, s);
    HIPCHK(hipMemcpyAsync(hp.data(), part, (size_t)nb * nblk * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.assign(nb, 0.0);
    for (int k = 0; k < nb; ++k) {
      for (int j = 0; j < nblk; ++j) out[k] += hp[(size_t)k * nblk + j];
      out[k] /= eref[hsl[k]];
    }
    return RBMC_OK;
  };
  // block-Jacobi energy error of every pair (the baseline of the ratios)
  std::vector<double> base_e(np_used, 0.0), be;
  for (int i0 = 0; i0 < (int)order.size(); i0 += B) {
    const int nb = std::min(B, (int)order.size() - i0);
    if ((st = batch_energy(order, i0, nb, false, false, be)) != RBMC_OK) return st;
    for (int k = 0; k < nb; ++k) base_e[order[i0 + k]] = be[k];
  }
  const int epochs = std::max(to->epochs, 0);
  const float lr = to->lr > 0.f ? to->lr : 1e-3f;
  int step = 0;
  std::vector<double> le;
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(fit.begin(), fit.end(), rng);
    double ep_err = 0.0, ep_base = 0.0;
    for (int i0 = 0; i0 + B <= n_fit; i0 += B) {
      if ((st = batch_energy(fit, i0, B, true, true, le)) != RBMC_OK) return st;
      for (int k = 0; k < B; ++k) {
        ep_err += le[k];
        ep_base += base_e[fit[i0 + k]];
      }
      // backward: layer l consumes a_{l-1} = relu(h_{l-1}) (the input for l = 0)
      const float* gout = gy;  // dL/d(output of layer l)
      for (int l = kNL - 1; l >= 0; --l) {
        const float* ain = (l == 0) ? bin : hs[l - 1];
        ConvWArgs wa{};
        wa.gout = gout;
        wa.ain = ain;
        wa.partial = wpart;
        wa.geom = g;
        wa.relu_in = l > 0;
        launch_conv3d_wgrad(wa, kCin[l], kCout[l], B, s);
        launch_sum_rows(wpart, wt_tiles * B, kCout[l] * kCin[l] * 27, m->lrn.g + kWOff[l], s);
        if (l > 0) {  // dL/dh_{l-1} = conv(gout, flipped W_l) * [h_{l-1} > 0]
          ConvArgs a{};
          a.in = gout;
          a.out = (gout == ga) ? gb : ga;
          a.w = m->lrn.wf + kWOff[l];
          a.mask = hs[l - 1];
          a.geom = g;
          a.scale = 1.f;
          launch_conv3d(a, kCout[l], kCin[l], B, s);
          gout = a.out;
        }
      }
      ++step;
      launch_adam(m->lrn.w, m->lrn.g, m->lrn.am, m->lrn.av, m->lrn.wb, kNW, lr, 0.9f, 0.999f,
                  1e-8f, step, s);
      for (int l = 0; l < kNL; ++l)
        launch_conv_wflip(m->lrn.wb + kWOff[l], kCin[l], kCout[l], m->lrn.wf + kWOff[l], s);
      HIPCHK(hipGetLastError());
    }
    if (loss_out) loss_out[ep] = (float)(ep_base > 0 ? ep_err / ep_base : 1.0);
  }
  // held-out energy error with the correction relative to block Jacobi alone
  double verr = 0.0, vbase = 0.0;
  for (int i0 = 0; i0 < n_val; i0 += B) {
    const int nb = std::min(B, n_val - i0);
    if ((st = batch_energy(val, i0, nb, true, false, le)) != RBMC_OK) return st;
    for (int k = 0; k < nb; ++k) {
      verr += le[k];
      vbase += base_e[val[i0 + k]];
    }
  }
  m->lrn.val_rel_err = vbase > 0.0 ? verr / vbase : 1.0;
  m->lrn.ready = true;
  m->lrn.usable = false;
  m->lrn.trial_bj = m->lrn.trial_lrn = -1;
  m->lrn.trial_s_bj = m->lrn.trial_s_lrn = -1.0;
  st = learned_rescale(m, su, 1.0 / su, s);  // fold the scales into the weights
  if (st != RBMC_OK) return st;
  if (m->lrn.val_rel_err < 1.0) {
    // acceptance trial on the held-out right-hand sides at the caller's
    // tolerance: the correction must save both iterations and time
    const HostCols hh = make_cols(ms, n_hold);
    st = ensure_ws(cx, ms, hh, false);
    if (st != RBMC_OK) return st;
    const double* zh = z + (size_t)c_hold * (n + (size_t)m->n_obs);
    rbmc_est_opts ot = *po;
    ot.n_samples = n_hold;
    ot.precond = RBMC_PC_BJ;
    // each run twice, the second timed (workspaces allocated, kernels loaded)
    rbmc_report rb{}, rl{};
    rbmc_status sb = RBMC_OK, sl = RBMC_OK;
    for (int k = 0; k < 2 && sb >= 0; ++k) sb = sample_set(cx, ms, hh, &ot, zh, cx->x, &rb, s);
    if (sb < 0) return sb;
    m->lrn.usable = true;
    ot.precond = RBMC_PC_BJ_LEARNED;
    for (int k = 0; k < 2 && sl >= 0; ++k) sl = sample_set(cx, ms, hh, &ot, zh, cx->x, &rl, s);
    m->lrn.usable = false;
    if (sl < 0) return sl;
    m->lrn.trial_bj = rb.pcg_it_max;
    m->lrn.trial_lrn = rl.pcg_it_max;
    m->lrn.trial_s_bj = rb.t_sample;
    m->lrn.trial_s_lrn = rl.t_sample;
    m->lrn.usable = sl == RBMC_OK && rl.pcg_it_max < rb.pcg_it_max && rl.t_sample < rb.t_sample;
  }
  if (loss_out) loss_out[epochs] = (float)m->lrn.val_rel_err;
  if (rep) {
    *rep = r1;
    rep->err_estimate = m->lrn.val_rel_err;
  }
  return RBMC_OK;
}

// ---------------------------------------------------------------------------
// Kronecker method for the subdomains (RBMC_SEL_KRON).  For A = [t0, t0 + T_A)
// x R the prior part of Q_AA is Q_t|A (x) Q_s|R, and the observations add a
// diagonal of rank n_o, so by the Woodbury identity
//   Q_AA^-1 = V (x) S^-1 - (V (x) S^-1) P Y P^T (V (x) S^-1),
//   S = Q_s|R,  V = (Q_t|A)^-1,  Y = (sigma^2 I + P^T (V (x) S^-1) P)^-1.
// S^-1 is formed once per spatial region (all time slabs of a tile share it),
// Y once per subdomain; the kernels in kernels_kron.hip turn them into the
// diagonal and stencil entries the estimator reads (Alg. 4, eq:hyperpar:4)
// and into the correction solves mu = Q_AA^-1 Q_AB x_B.
// ---------------------------------------------------------------------------
struct Carve {  // bump allocation inside one device block (256-byte aligned)
  char* base = nullptr;
  size_t off = 0;
  double* d(size_t n) {
    off = (off + 255) / 256 * 256;
    double* p = (double*)(base + off);
    off += n * 8;
    return p;
  }
};

// Sweep workspaces of a Gauss-Jordan inversion of order np (see InvJob).
void carve_gj(Carve& cv, int np, InvJob& j) {
  const size_t w = sweep_width_of(np);
  j.B = cv.d((size_t)np * w);
  j.U = cv.d((size_t)np * w);
  j.P = cv.d(w * w);
  j.B2 = cv.d(w * 128);
  j.U2 = cv.d(w * 128);
  j.P2 = cv.d((size_t)128 * 128);
}

rbmc_status ensure_kws(rbmc_ctx* cx, size_t bytes) {
  if (cx->kws_cap >= bytes) return RBMC_OK;
  cx->kws.release();
  cx->kws_base = nullptr;
  cx->kws_cap = 0;
  HIPCHK(cx->kws.alloc((void**)&cx->kws_base, bytes));
  cx->kws_cap = bytes;
  return RBMC_OK;
}

// Observed slots of every subdomain (plan and mask only), the regions'
// S^-1 storage and K in the 13-point coefficient layout.
rbmc_status kron_static(rbmc_model* m) {
  if (m->kron_static) return RBMC_OK;
  const Plan& P = m->plan;
  hipStream_t s = m->ctx->stream;
  m->kreg_of.assign(P.regions.size(), -1);
  m->ksub.clear();
  m->kreg.clear();
  std::vector<int> idx;  // all index tables of the model, one upload
  std::vector<size_t> at;
  for (size_t c = 0; c < P.sub.size(); ++c) {
    const Chain& ch = P.sub[c];
    const Region& g = P.regions[ch.region];
    if (m->kreg_of[ch.region] < 0) {
      rbmc_model::KronReg r;
      r.region = ch.region;
      r.nb = g.nb();
      r.np = pad_to(r.nb);
      HIPCHK(m->kpool.alloc((void**)&r.inv, (size_t)r.np * r.np * 8));
      HIPCHK(m->kpool.alloc((void**)&r.dR, (size_t)r.np * 8));
      HIPCHK(m->kpool.alloc((void**)&r.qR, (size_t)r.np * 8));
      HIPCHK(m->kpool.alloc((void**)&r.kR, (size_t)r.np * 8));
      std::vector<char> in_r((size_t)P.ns, 0);
      for (int a = 0; a < g.nb(); ++a) in_r[g.nodes[a]] = 1;
      std::vector<int> ring;
      for (int a = 0; a < g.nb(); ++a) {
        const int x = g.nodes[a] % P.mx, y = g.nodes[a] / P.mx;
        bool rim = false;
        for (int dy = -2; dy <= 2 && !rim; ++dy)
          for (int dx = -2; dx <= 2 && !rim; ++dx) {
            if (std::abs(dx) + std::abs(dy) > 2) continue;
            const int xx = x + dx, yy = y + dy;
            rim = xx >= 0 && xx < P.mx && yy >= 0 && yy < P.my && !in_r[(size_t)yy * P.mx + xx];
          }
        if (rim) ring.push_back(a);
      }
      for (int c0 = 0; c0 < g.nb(); c0 += 256) {
        int lo = INT_MAX, hi = -1;
        for (int a = c0; a < std::min(c0 + 256, g.nb()); ++a)
          if (g.in_box[a])
            for (int q = 0; q < kNS; ++q) {
              const int c = g.nbr[(size_t)a * kNS + q];
              if (c >= 0) {
                lo = std::min(lo, c);
                hi = std::max(hi, c);
              }
            }
        if (hi >= lo) r.mc_win = std::max(r.mc_win, hi - lo + 1);
      }
      r.nring = (int)ring.size();
      r.nrp = r.nring > 0 ? pad_to(r.nring) : 0;
      r.rim = r.nrp < r.np;  // the rim products pay only when the rim is a part of R
      if (r.rim && r.nring > 0) {
        ring.resize(r.nrp, -1);
        HIPCHK(m->kpool.alloc((void**)&r.d_ring, (size_t)r.nrp * 4));
        HIPCHK(hipMemcpyAsync(r.d_ring, ring.data(), (size_t)r.nrp * 4, hipMemcpyHostToDevice,
                              s));
        HIPCHK(m->kpool.alloc((void**)&r.rinv, (size_t)r.np * r.nrp * 8));
        HIPCHK(hipStreamSynchronize(s));  // ring is host memory of this scope
      } else if (!r.rim) {
        r.nring = r.nrp = 0;
      }
      m->kreg_of[ch.region] = (int)m->kreg.size();
      m->kreg.push_back(r);
    }
    rbmc_model::KronSub k;
    k.chain = (int)c;
    k.TA = ch.T;
    std::vector<int> oa, ot;
    for (int t = 0; t < ch.T; ++t) {
      k.goff.push_back((int)oa.size());
      int cnt = 0;
      for (int a = 0; a < g.nb(); ++a)
        if (m->mask[(size_t)(ch.t0 + t) * P.ns + g.nodes[a]]) {
          oa.push_back(a);
          ot.push_back(t);
          ++cnt;
        }
      const int pad = (cnt + 15) / 16 * 16;
      for (int i = cnt; i < pad; ++i) {
        oa.push_back(-1);
        ot.push_back(t);
      }
      k.gpad.push_back(pad);
      k.nobs += cnt;
    }
    k.nc = std::max(kPad, pad_to((int)oa.size()));
    while ((int)oa.size() < k.nc) {  // trailing unused slots (in no group)
      oa.push_back(-1);
      ot.push_back(0);
    }
    at.push_back(idx.size());
    idx.insert(idx.end(), oa.begin(), oa.end());
    idx.insert(idx.end(), ot.begin(), ot.end());
    idx.insert(idx.end(), k.goff.begin(), k.goff.end());
    idx.insert(idx.end(), k.gpad.begin(), k.gpad.end());
    m->ksub.push_back(std::move(k));
  }
  int* d_idx = nullptr;
  HIPCHK(m->kpool.alloc((void**)&d_idx, std::max<size_t>(idx.size(), 1) * 4));
  HIPCHK(hipMemcpyAsync(d_idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, s));
  for (size_t c = 0; c < m->ksub.size(); ++c) {
    rbmc_model::KronSub& k = m->ksub[c];
    k.d_obs_a = d_idx + at[c];
    k.d_obs_t = k.d_obs_a + k.nc;
    k.d_goff = k.d_obs_t + k.nc;
    k.d_gpad = k.d_goff + k.TA;
  }
  std::vector<double> kk13((size_t)kNS * P.ns, 0.0);
  std::copy(m->co.kk.begin(), m->co.kk.end(), kk13.begin());
  HIPCHK(m->kpool.alloc((void**)&m->d_kk13, kk13.size() * 8));
  HIPCHK(hipMemcpyAsync(m->d_kk13, kk13.data(), kk13.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  m->kron_static = true;
  return RBMC_OK;
}

// (Q_t restricted to steps [t0, t0 + TA))^-1, TA x TA, symmetric: each column
// by a tridiagonal elimination, then the two triangles averaged.
std::vector<double> time_inverse(const Coefs& co, int t0, int TA) {
  std::vector<double> V((size_t)TA * TA, 0.0), cp(TA), dp(TA);
  const double a = co.qo;
  for (int j = 0; j < TA; ++j) {
    for (int t = 0; t < TA; ++t) {
      const double b = co.qd[t0 + t];
      const double den = t == 0 ? b : b - a * cp[t - 1];
      cp[t] = a / den;
      const double rhs = (t == j) ? 1.0 : 0.0;
      dp[t] = (t == 0 ? rhs : rhs - a * dp[t - 1]) / den;
    }
    double y = dp[TA - 1];
    V[(size_t)(TA - 1) * TA + j] = y;
    for (int t = TA - 2; t >= 0; --t) {
      y = dp[t] - cp[t] * y;
      V[(size_t)t * TA + j] = y;
    }
  }
  for (int i = 0; i < TA; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (V[(size_t)i * TA + j] + V[(size_t)j * TA + i]);
      V[(size_t)i * TA + j] = V[(size_t)j * TA + i] = v;
    }
  return V;
}

// S^-1 = (Q_s|R)^-1 of every region of the models that need it (after a
// change of theta), with the node quantities dR, qR, kR.
rbmc_status kron_regions(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, hipStream_t s,
                         rbmc_report* rep) {
  std::vector<std::pair<rbmc_model*, int>> todo;
  for (rbmc_model* m : ms)
    if (!m->kron_ready)
      for (size_t r = 0; r < m->kreg.size(); ++r) todo.push_back({m, (int)r});
  if (todo.empty()) return RBMC_OK;
  size_t bytes = 4096;
  for (auto& tr : todo) {
    const int np = tr.first->kreg[tr.second].np;
    const size_t w = sweep_width_of(np);
    bytes += (2 * (size_t)np * w + w * w + 2 * w * 128 + 128 * 128) * 8 + 6 * 256;
  }
  // one info flag per region job, at the start of the workspace
  bytes += todo.size() * 4 + 256;
  rbmc_status st = ensure_kws(cx, bytes);
  if (st != RBMC_OK) return st;
  Carve cv{cx->kws_base, 0};
  int* info = (int*)cv.d((todo.size() + 1) / 2);
  HIPCHK(hipMemsetAsync(info, 0, todo.size() * 4, s));
  Arena& ar = cx->arenaB;
  ar.clear();
  Program pg;
  StencilList sl;
  std::vector<InvJob> jobs;
  TileList<KronRegionTask> rt;
  TileList<KronBuildTask> gt;
  for (size_t i = 0; i < todo.size(); ++i) {
    rbmc_model* m = todo[i].first;
    const rbmc_model::KronReg& R = m->kreg[todo[i].second];
    StencilTask t{};
    t.rg = m->d_regions + R.region;
    t.qs = m->d_qs;
    t.ns = m->plan.ns;
    t.M = nullptr;
    t.alpha = 0.0;
    t.gamma = 1.0;
    t.pad_identity = 1;
    t.out = R.inv;
    t.ldout = R.np;
    t.ldm = R.np;
    t.ncols = R.np;
    sl.add(t, R.np, R.nb);
    InvJob j{};
    j.M = R.inv;
    j.np = R.np;
    j.nb = R.nb;
    j.info = info + i;
    j.base = 0;
    carve_gj(cv, R.np, j);
    jobs.push_back(j);
    KronRegionTask k{};
    k.inv = R.inv;
    k.rg = t.rg;
    k.dm = m->d_dm;
    k.dR = R.dR;
    k.qR = R.qR;
    k.kR = R.kR;
    rt.add(k, (R.np + 255) / 256);
    if (R.rinv) {  // S^-1[:, rim]
      KronBuildTask g{};
      g.mode = 0;
      g.inv = R.inv;
      g.obs_a = R.d_ring;
      g.np = R.np;
      g.nc = R.nrp;
      g.out = R.rinv;
      gt.add(g, kron_cols_tiles(R.np, R.nrp), 16.0 * R.np * R.nrp);
    }
  }
  pg.stencil(ar, sl);
  pg.inverse(ar, jobs);
  pg.kron(ar, 14, rt);
  pg.kron(ar, 15, gt);
  HIPCHK(ar.upload(s));
  st = run(cx, pg, s, ar);
  if (st != RBMC_OK) return st;
  std::vector<int> hinfo(todo.size());
  HIPCHK(hipMemcpyAsync(hinfo.data(), info, todo.size() * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (size_t i = 0; i < todo.size(); ++i)
    if (hinfo[i] != 0) {
      if (rep) rep->fail_block = hinfo[i] - 1;
      return fail(RBMC_E_NOT_SPD, "spatial block Q_s|R of region " +
                                      std::to_string(todo[i].second) + " lost positive definiteness");
    }
  for (rbmc_model* m : ms) m->kron_ready = true;
  return RBMC_OK;
}

// Device workspace of one subdomain in a batch (bytes, with alignment slack).
size_t kron_sub_bytes(const rbmc_model* m, const rbmc_model::KronSub& k, int nk) {
  const rbmc_model::KronReg& R = m->kreg[m->kreg_of[m->plan.sub[k.chain].region]];
  const size_t np = R.np, nc = k.nc, TA = k.TA, w = sweep_width_of(k.nc);
  size_t d = 3 * np * nc + nc * nc + TA * TA * 3 * np + TA * TA;  // Z, KZ, X, C, part, V
  d += 2 * nc * w + w * w + 2 * w * 128 + 128 * 128;              // inversion of C
  if (nk > 0) d += 2 * np * TA * nk + 2 * nc * nk + (size_t)R.nrp * TA * nk;  // Rb Ub v w Rc
  return d * 8 + 21 * 256;
}

struct KronBuf {
  double *Z, *KZ, *X, *C, *part, *V, *Rb, *Ub, *v, *w, *Rc;
  InvJob inv;
};

// The subdomains of a set, in order: (model index, subdomain index).
std::vector<std::pair<int, int>> kron_refs(const std::vector<rbmc_model*>& ms) {
  std::vector<std::pair<int, int>> r;
  for (size_t j = 0; j < ms.size(); ++j)
    for (size_t c = 0; c < ms[j]->ksub.size(); ++c) r.push_back({(int)j, (int)c});
  return r;
}

// Selected entries of one batch of subdomains [i0, i1) of refs.
rbmc_status kron_det_batch(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms,
                           const std::vector<std::pair<int, int>>& refs, size_t i0, size_t i1,
                           const std::vector<KronBuf>& kb, const EstLayout& L,
                           const std::vector<size_t>& lidx,
                           const std::vector<double*>& diag_out, hipStream_t s,
                           rbmc_report* rep) {
  Arena& ar = cx->arenaB;
  ar.clear();
  Program pg;
  TileList<KronBuildTask> zt, ct;
  StencilList kz;
  std::vector<InvJob> jobs;
  int maxTA = 0;
  for (size_t i = i0; i < i1; ++i) {
    rbmc_model* m = ms[refs[i].first];
    const rbmc_model::KronSub& k = m->ksub[refs[i].second];
    const Chain& ch = m->plan.sub[k.chain];
    const rbmc_model::KronReg& R = m->kreg[m->kreg_of[ch.region]];
    const KronBuf& b = kb[i - i0];
    maxTA = std::max(maxTA, k.TA);
    pg.fill(b.part, (size_t)k.TA * k.TA * 3 * R.np);
    KronBuildTask t{};
    t.mode = 0;
    t.inv = R.inv;
    t.Z = b.Z;
    t.V = b.V;
    t.obs_a = k.d_obs_a;
    t.obs_t = k.d_obs_t;
    t.np = R.np;
    t.nc = k.nc;
    t.TA = k.TA;
    t.noise = 1.0 / m->co.dobs;
    t.out = b.Z;
    zt.add(t, kron_cols_tiles(R.np, k.nc), 16.0 * R.np * k.nc);
    t.mode = 1;
    t.out = b.C;
    ct.add(t, kron_cols_tiles(k.nc, k.nc), 16.0 * k.nc * k.nc);
    StencilTask st{};
    st.rg = m->d_regions + ch.region;
    st.qs = m->d_kk13;
    st.ns = m->plan.ns;
    st.M = b.Z;
    st.ldm = R.np;
    st.alpha = 1.0;
    st.out = b.KZ;
    st.ldout = R.np;
    st.ncols = k.nc;
    kz.add(st, R.np, R.nb);
    InvJob j = b.inv;
    j.M = b.C;
    j.np = k.nc;
    j.nb = k.nobs;
    j.info = m->d_info + m->plan.bj.size() + k.chain;
    j.base = 0;
    jobs.push_back(j);
  }
  pg.kron(ar, 15, zt);
  pg.stencil(ar, kz);
  pg.kron(ar, 15, ct);
  pg.inverse(ar, jobs);
  for (int g = 0; g < maxTA; ++g) {
    GemmList gx;
    TileList<KronReduceTask> rl;
    for (size_t i = i0; i < i1; ++i) {
      rbmc_model* m = ms[refs[i].first];
      const rbmc_model::KronSub& k = m->ksub[refs[i].second];
      if (g >= k.TA || k.gpad[g] == 0) continue;
      const rbmc_model::KronReg& R = m->kreg[m->kreg_of[m->plan.sub[k.chain].region]];
      const KronBuf& b = kb[i - i0];
      // X_g = Z_g Y_{g,:}  (np x nc, K = the group's slots)
      gx.add(b.Z + (size_t)k.goff[g] * R.np, b.C + k.goff[g], nullptr, b.X, R.np, k.nc, k.gpad[g],
             R.np, k.nc, R.np, 1.0, 0.0, 0, 0, R.nb, k.gpad[g]);
      KronReduceTask rt{};
      rt.X = b.X;
      rt.Z = b.Z;
      rt.KZ = b.KZ;
      rt.obs_a = k.d_obs_a;
      rt.goff = k.d_goff;
      rt.gpad = k.d_gpad;
      rt.part = b.part;
      rt.np = R.np;
      rt.TA = k.TA;
      rt.g = g;
      rl.add(rt, (R.np + 63) / 64, 24.0 * R.np * k.nc);
    }
    pg.gemm(ar, gx);
    pg.kron(ar, 16, rl, RBMC_KF_KRON_REDUCE);
  }
  TileList<KronDetTask> dt;
  for (size_t i = i0; i < i1; ++i) {
    rbmc_model* m = ms[refs[i].first];
    const rbmc_model::KronSub& k = m->ksub[refs[i].second];
    const Chain& ch = m->plan.sub[k.chain];
    const rbmc_model::KronReg& R = m->kreg[m->kreg_of[ch.region]];
    const KronBuf& b = kb[i - i0];
    const size_t c = lidx[i];
    for (int t = ch.ct0 - ch.t0; t < ch.ct0 - ch.t0 + ch.cT; ++t) {
      KronDetTask d{};
      d.V = b.V;
      d.part = b.part;
      d.dR = R.dR;
      d.qR = R.qR;
      d.kR = R.kR;
      d.rg = m->d_regions + ch.region;
      d.dm = m->d_dm;
      d.diag_out = diag_out[refs[i].first];
      d.partial = cx->epart;
      d.out_index = (int)L.det_index(c, t, 0);
      d.nchk = (int)L.nchk(c);
      d.TA = k.TA;
      d.t = t;
      d.t0 = ch.t0;
      dt.add(d, (int)L.nchk(c));
    }
  }
  pg.kron(ar, 17, dt);
  // info flags of the batch's capacitance inversions start at zero
  for (size_t i = i0; i < i1; ++i) {
    rbmc_model* m = ms[refs[i].first];
    HIPCHK(hipMemsetAsync(m->d_info + m->plan.bj.size() + m->ksub[refs[i].second].chain, 0, 4, s));
  }
  HIPCHK(ar.upload(s));
  rbmc_status st = run(cx, pg, s, ar);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  for (size_t i = i0; i < i1; ++i) {
    rbmc_model* m = ms[refs[i].first];
    const int c = m->ksub[refs[i].second].chain;
    int v = 0;
    HIPCHK(hipMemcpy(&v, m->d_info + m->plan.bj.size() + c, 4, hipMemcpyDeviceToHost));
    if (v != 0) {
      if (rep) {
        rep->fail_subdomain = c;
        rep->fail_block = v - 1;
      }
      return fail(RBMC_E_NOT_SPD, "capacitance matrix of subdomain " + std::to_string(c) +
                                      " lost positive definiteness");
    }
  }
  return RBMC_OK;
}

// Correction solves and Monte Carlo sums of one batch (samples x at x_base in
// the column layout h, nk of them).
// gather_z: form Z = S^-1[:, a_o] first (a pass after the first, whose Z
// went with the batch's deterministic part); scale = 1 / (total samples),
// accum: add to the Monte Carlo sums of earlier passes.
rbmc_status kron_corr_batch(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms, const HostCols& h,
                            int nk, const double* x_base,
                            const std::vector<std::pair<int, int>>& refs, size_t i0, size_t i1,
                            const std::vector<KronBuf>& kb, const EstLayout& L,
                            const std::vector<size_t>& lidx,
                            const std::vector<double*>& diag_out, int mixed, bool gather_z,
                            double scale, int accum, hipStream_t s) {
  Arena& ar = cx->arenaB;
  ar.clear();
  Program pg;
  if (gather_z) {
    TileList<KronBuildTask> zt;
    for (size_t i = i0; i < i1; ++i) {
      rbmc_model* m = ms[refs[i].first];
      const rbmc_model::KronSub& k = m->ksub[refs[i].second];
      const rbmc_model::KronReg& R = m->kreg[m->kreg_of[m->plan.sub[k.chain].region]];
      KronBuildTask t{};
      t.mode = 0;
      t.inv = R.inv;
      t.obs_a = k.d_obs_a;
      t.obs_t = k.d_obs_t;
      t.np = R.np;
      t.nc = k.nc;
      t.TA = k.TA;
      t.out = kb[i - i0].Z;
      zt.add(t, kron_cols_tiles(R.np, k.nc), 16.0 * R.np * k.nc);
    }
    pg.kron(ar, 15, zt);
  }
  TileList<PanelTask> rt;
  TileList<PanelTask> bt[2];                        // separator terms (first, last step)
  std::vector<std::pair<double*, size_t>> uz;       // U blocks that are zero (empty rim)
  GemmList gu, gw, gz;
  gu.mixed = gw.mixed = gz.mixed = mixed;
  TileList<KronMixTask> m1, m2;
  TileList<KronObsTask> ob;
  TileList<McTask> mt, mt2;
  for (size_t i = i0; i < i1; ++i) {
    const int j = refs[i].first;
    rbmc_model* m = ms[j];
    const rbmc_model::KronSub& k = m->ksub[refs[i].second];
    const Chain& ch = m->plan.sub[k.chain];
    const rbmc_model::KronReg& R = m->kreg[m->kreg_of[ch.region]];
    const KronBuf& b = kb[i - i0];
    const size_t panel = (size_t)R.np * nk;
    // U = S^-1 r, r = Q_AB x_B one panel per step (panels are stacked
    // columns).  With the rim products: r = r~ + (Q_t)_{t,t'} S x_t'|R, where
    // r~ (spatial neighbours outside R) lives on the rim of R and the second
    // term appears only at a step next to the time separator (t' outside the
    // chain), so U = S^-1[:, rim] r~|rim + (Q_t)_{t,t'} x_t'|R.
    if (R.rim) {
      for (int t = 0; t < k.TA && R.nring > 0; ++t) {
        PanelTask pt{};
        pt.P = b.Rc + (size_t)t * R.nrp * nk;
        pt.rg = m->d_regions + ch.region;
        pt.dm = m->d_dm;
        pt.X = x_base + h.base[j];
        pt.n_k = nk;
        pt.t = ch.t0 + t;
        pt.t0 = ch.t0;
        pt.T = ch.T;
        pt.mode = 3;
        pt.rows = R.d_ring;
        pt.ld = R.nrp;
        rt.add(pt, panel_tiles(R.nrp, nk), 16.0 * R.nring * nk);
      }
      if (R.nring > 0)
        gu.add(R.rinv, b.Rc, nullptr, b.Ub, R.np, k.TA * nk, R.nrp, R.np, R.nrp, R.np, 1.0, 0.0,
               0, 0, R.nb, R.nring);
      else
        uz.push_back({b.Ub, (size_t)R.np * k.TA * nk});
      // the separator steps t0 - 1 and t0 + TA (inside the domain)
      for (int side = 0; side < 2; ++side) {
        const int t = side == 0 ? 0 : k.TA - 1;
        const int tg = side == 0 ? ch.t0 - 1 : ch.t0 + k.TA;
        if (tg < 0 || tg >= m->plan.T) continue;
        PanelTask pt{};
        pt.P = b.Ub + (size_t)t * panel;
        pt.rg = m->d_regions + ch.region;
        pt.dm = m->d_dm;
        pt.X = x_base + h.base[j];
        pt.n_k = nk;
        pt.t = tg;
        pt.mode = 4;
        pt.w = m->co.qo;
        bt[side].add(pt, panel_tiles(R.np, nk), 24.0 * R.nb * nk);
      }
    } else {
      for (int t = 0; t < k.TA; ++t) {
        PanelTask pt{};
        pt.P = b.Rb + (size_t)t * panel;
        pt.rg = m->d_regions + ch.region;
        pt.dm = m->d_dm;
        pt.X = x_base + h.base[j];
        pt.n_k = nk;
        pt.t = ch.t0 + t;
        pt.t0 = ch.t0;
        pt.T = ch.T;
        pt.mode = 2;
        rt.add(pt, panel_tiles(R.np, nk), 16.0 * R.nb * nk);
      }
      gu.add(R.inv, b.Rb, nullptr, b.Ub, R.np, k.TA * nk, R.np, R.np, R.np, R.np, 1.0, 0.0, 0, 0,
             R.nb, R.nb);
    }
    KronMixTask mx{};
    mx.V = b.V;
    mx.U = b.Ub;
    mx.In = nullptr;
    mx.out = b.Rb;
    mx.np = R.np;
    mx.n_k = nk;
    mx.TA = k.TA;
    mx.alpha = 1.0;
    mx.beta = 0.0;
    m1.add(mx, kron_mix_tiles(R.np, nk), 16.0 * R.nb * nk * k.TA);
    KronObsTask ot{};
    ot.U = b.Rb;
    ot.v = b.v;
    ot.obs_a = k.d_obs_a;
    ot.obs_t = k.d_obs_t;
    ot.np = R.np;
    ot.nc = k.nc;
    ot.n_k = nk;
    ob.add(ot, kron_cols_tiles(k.nc, nk));
    gw.add(b.C, b.v, nullptr, b.w, k.nc, nk, k.nc, k.nc, k.nc, k.nc, 1.0, 0.0, 0, 0, k.nobs,
           k.nobs);
    for (int g = 0; g < k.TA; ++g)
      if (k.gpad[g] > 0)
        gz.add(b.Z + (size_t)k.goff[g] * R.np, b.w + k.goff[g], nullptr, b.Ub + (size_t)g * panel,
               R.np, nk, k.gpad[g], R.np, k.nc, R.np, 1.0, 0.0, 0, 0, R.nb, k.gpad[g]);
    mx.U = b.Ub;
    mx.In = b.Rb;
    mx.out = b.Rb;
    mx.alpha = -1.0;
    mx.beta = 1.0;
    m2.add(mx, kron_mix_tiles(R.np, nk), 24.0 * R.nb * nk * k.TA);
    const size_t c = lidx[i];
    // several core steps per task when their windows fit in LDS
    const int S = R.mc_win > 0
                      ? std::max(1, std::min(mc_max_steps(), mc_lds_doubles() / R.mc_win - 2))
                      : 1;
    const int tc0 = ch.ct0 - ch.t0, tc1 = tc0 + ch.cT;
    for (int t = tc0; S > 1 && t < tc1; t += S) {
      McTask q{};
      q.stack = b.Rb;
      q.ta = k.TA;
      q.tl = t;
      q.steps = std::min(S, tc1 - t);
      q.np = R.np;
      q.rg = m->d_regions + ch.region;
      q.dm = m->d_dm;
      q.diag_out = diag_out[j];
      q.partial = cx->epart + L.det_len;
      q.out_index = (int)L.mc_index(c, t);
      q.n_k = nk;
      q.scale = scale;
      q.accum = accum;
      q.t = ch.t0 + t;
      mt2.add(q, mc_chunks(R.np), 8.0 * R.nb * nk * q.steps);
    }
    for (int t = tc0; S == 1 && t < tc1; ++t) {
      McTask q{};
      q.mu[0] = t - 1 >= 0 ? b.Rb + (size_t)(t - 1) * panel : nullptr;
      q.mu[1] = b.Rb + (size_t)t * panel;
      q.mu[2] = t + 1 < k.TA ? b.Rb + (size_t)(t + 1) * panel : nullptr;
      q.np = R.np;
      q.rg = m->d_regions + ch.region;
      q.dm = m->d_dm;
      q.diag_out = diag_out[j];
      q.partial = cx->epart + L.det_len;
      q.out_index = (int)L.mc_index(c, t);
      q.n_k = nk;
      q.scale = scale;
      q.accum = accum;
      q.t = ch.t0 + t;
      mt.add(q, mc_chunks(R.np), 8.0 * R.nb * nk);
    }
  }
  pg.panels(ar, rt);
  for (const auto& z : uz) pg.fill(z.first, z.second);
  pg.gemm(ar, gu);
  pg.panels(ar, bt[0]);  // two launches: a one-step chain takes both terms
  pg.panels(ar, bt[1]);
  pg.kron(ar, 18, m1, RBMC_KF_TMIX);
  pg.kron(ar, 19, ob);
  pg.gemm(ar, gw);
  // the products Z_g w_g overwrite the panel of every step with observations;
  // the others must be zero
  for (size_t i = i0; i < i1; ++i) {
    rbmc_model* m = ms[refs[i].first];
    const rbmc_model::KronSub& k = m->ksub[refs[i].second];
    const rbmc_model::KronReg& R = m->kreg[m->kreg_of[m->plan.sub[k.chain].region]];
    const size_t panel = (size_t)R.np * nk;
    for (int g = 0; g < k.TA; ++g)
      if (k.gpad[g] == 0) pg.fill(kb[i - i0].Ub + (size_t)g * panel, panel);
  }
  pg.gemm(ar, gz);
  pg.kron(ar, 18, m2, RBMC_KF_TMIX);
  pg.mc(ar, mt);
  pg.mc(ar, mt2, true);
  HIPCHK(ar.upload(s));
  rbmc_status st = run(cx, pg, s, ar);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  return RBMC_OK;
}

// Samples of pass c of a chunked estimate: columns [k0, k0 + kn) of every
// model in the column layout *h, at *x.
using KronSampler =
    std::function<rbmc_status(int k0, int kn, const double** x, HostCols* h, rbmc_report* r)>;

// Device workspace of one subdomain in a pass after the first (Z, V and the
// correction buffers; Y is in the bank).
size_t kron_corr_bytes(const rbmc_model* m, const rbmc_model::KronSub& k, int nk) {
  const rbmc_model::KronReg& R = m->kreg[m->kreg_of[m->plan.sub[k.chain].region]];
  const size_t np = R.np, nc = k.nc, TA = k.TA;
  return (np * nc + TA * TA + 2 * np * TA * nk + 2 * nc * nk + (size_t)R.nrp * TA * nk) * 8 +
         11 * 256;
}

// The estimator by the Kronecker method, over batches of subdomains sized to
// the free device memory.  Samples: x_given (layout *h_given, nk_total
// columns) or, when sampler is set, passes of `chunk` columns drawn by it.
// With one pass every batch forms its selected entries and corrects its
// subdomains in turn; with several, the selected entries come first (Y of
// every subdomain kept in the bank), then each pass draws its samples and
// corrects all batches, adding to the Monte Carlo sums.
rbmc_status estimate_set_kron(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms,
                              const rbmc_est_opts* o, int nk_total, int chunk,
                              const KronSampler& sampler, const double* x_given,
                              const HostCols* h_given, const std::vector<double*>& diag_out,
                              const std::vector<double*>& trace_out, rbmc_report* rep) {
  g_tune = cx->tune;
  const int mixed = o->precision == RBMC_MIXED;
  {
    rbmc_status e = sep_check(ms, o);
    if (e != RBMC_OK) return e;
  }
  hipStream_t s = cx->stream;
  const int npass = nk_total > 0 ? (nk_total + chunk - 1) / chunk : 0;
  double t_fac = 0.0, t_cor = 0.0, t_smp = 0.0, ta = now_s();
  rbmc_status st = RBMC_OK, st_s = RBMC_OK;
  for (rbmc_model* m : ms) {
    st = kron_static(m);
    if (st != RBMC_OK) return st;
  }
  const std::vector<std::pair<int, int>> refs = kron_refs(ms);
  EstLayout L;
  std::vector<size_t> lidx;
  for (const auto& r : refs) {
    rbmc_model* m = ms[r.first];
    const Chain& ch = m->plan.sub[m->ksub[r.second].chain];
    lidx.push_back(L.ch.size());
    L.add(ch, m, m->kreg[m->kreg_of[ch.region]].np, r.first);
  }
  L.finish();
  st = ensure_epart(cx, L);
  if (st != RBMC_OK) return st;
  launch_fill(cx->epart, L.det_len + L.mc_len, 0.0, s);
  // sampler report, summed over passes
  int it_max = 0;
  double it_sum = 0.0, res_max = 0.0;
  auto draw = [&](int k0, int kn, const double** x, HostCols* hc) -> rbmc_status {
    rbmc_report r{};
    const double t = now_s();
    rbmc_status e = sampler(k0, kn, x, hc, &r);
    t_smp += now_s() - t;
    if (e < 0) return e;
    if (e != RBMC_OK) st_s = e;
    it_max = std::max(it_max, r.pcg_it_max);
    it_sum += r.pcg_it_mean * kn;
    res_max = std::max(res_max, r.max_rel_residual);
    return RBMC_OK;
  };
  // the first pass is drawn before the batches are sized (its workspace must
  // fit beside them); with one pass its samples are corrected batch by batch
  // together with the selected entries
  const double* x1 = x_given;
  HostCols h1;
  if (npass >= 1 && sampler) {
    st = draw(0, std::min(chunk, nk_total), &x1, &h1);
    if (st != RBMC_OK) return st;
  } else if (x_given) {
    h1 = *h_given;
  }
  ta = now_s();
  st = kron_regions(cx, ms, s, rep);
  if (st != RBMC_OK) return st;
  // several passes: Y of every subdomain and the deterministic diagonals in the bank
  std::vector<double*> ybank(refs.size(), nullptr), ddet(ms.size(), nullptr);
  if (npass > 1) {
    size_t need = 0;
    for (const auto& r : refs) {
      const size_t nc = ms[r.first]->ksub[r.second].nc;
      need += nc * nc * 8 + 256;
    }
    for (rbmc_model* m : ms) need += (size_t)m->plan.n * 8 + 256;
    if (cx->kbank_cap < need) {  // a larger bank: it comes first, batches take what is left
      cx->kws.release();
      cx->kws_base = nullptr;
      cx->kws_cap = 0;
      cx->kbank.release();
      cx->kbank_base = nullptr;
      cx->kbank_cap = 0;
      HIPCHK(cx->kbank.alloc((void**)&cx->kbank_base, need));
      cx->kbank_cap = need;
    }
    Carve cb{cx->kbank_base, 0};
    for (size_t i = 0; i < refs.size(); ++i) {
      const size_t nc = ms[refs[i].first]->ksub[refs[i].second].nc;
      ybank[i] = cb.d(nc * nc);
    }
    for (size_t j = 0; j < ms.size(); ++j) ddet[j] = cb.d((size_t)ms[j]->plan.n);
  }
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const size_t reserve = ((size_t)1 << 30) + total_b / 64;
  size_t avail = free_b + cx->kws_cap > reserve ? free_b + cx->kws_cap - reserve : 0;
  if (cx->kron_batch_cap > 0) avail = std::min(avail, cx->kron_batch_cap);
  t_fac += now_s() - ta;
  // batches [i0, i1) of refs whose workspace fits
  auto next_batch = [&](size_t i0, bool corr_only, int nk) {
    size_t i1 = i0, bytes = 0;
    while (i1 < refs.size()) {
      const rbmc_model* m = ms[refs[i1].first];
      const rbmc_model::KronSub& k = m->ksub[refs[i1].second];
      const size_t b = corr_only ? kron_corr_bytes(m, k, nk) : kron_sub_bytes(m, k, nk);
      if (i1 > i0 && bytes + b > avail) break;
      bytes += b;
      ++i1;
    }
    return std::make_pair(i1, bytes);
  };
  // carve a batch; V of each subdomain uploaded
  auto carve_batch = [&](size_t i0, size_t i1, bool corr_only, int nk,
                         std::vector<KronBuf>& kb) -> rbmc_status {
    Carve cv{cx->kws_base, 0};
    kb.assign(i1 - i0, KronBuf{});
    std::vector<double> hV;
    std::vector<size_t> vat;
    for (size_t i = i0; i < i1; ++i) {
      rbmc_model* m = ms[refs[i].first];
      const rbmc_model::KronSub& k = m->ksub[refs[i].second];
      const Chain& ch = m->plan.sub[k.chain];
      const int np = m->kreg[m->kreg_of[ch.region]].np;
      KronBuf& b = kb[i - i0];
      b.Z = cv.d((size_t)np * k.nc);
      b.V = cv.d((size_t)k.TA * k.TA);
      if (!corr_only) {
        b.KZ = cv.d((size_t)np * k.nc);
        b.X = cv.d((size_t)np * k.nc);
        b.part = cv.d((size_t)k.TA * k.TA * 3 * np);
        b.C = npass > 1 ? ybank[i] : cv.d((size_t)k.nc * k.nc);
        carve_gj(cv, k.nc, b.inv);
      } else {
        b.C = ybank[i];
      }
      if (nk > 0 && (corr_only || npass == 1)) {
        b.Rb = cv.d((size_t)np * k.TA * nk);
        b.Ub = cv.d((size_t)np * k.TA * nk);
        b.v = cv.d((size_t)k.nc * nk);
        b.w = cv.d((size_t)k.nc * nk);
        const int nrp = m->kreg[m->kreg_of[ch.region]].nrp;
        b.Rc = nrp > 0 ? cv.d((size_t)nrp * k.TA * nk) : nullptr;
      }
      const std::vector<double> V = time_inverse(m->co, ch.t0, k.TA);
      vat.push_back(hV.size());
      hV.insert(hV.end(), V.begin(), V.end());
    }
    for (size_t i = i0; i < i1; ++i) {
      const size_t len = (i + 1 < i1 ? vat[i + 1 - i0] : hV.size()) - vat[i - i0];
      HIPCHK(hipMemcpyAsync(kb[i - i0].V, hV.data() + vat[i - i0], len * 8,
                            hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));  // hV is host memory of this scope
    return RBMC_OK;
  };
  const int nk1 = npass == 1 ? nk_total : 0;  // samples corrected with the selected entries
  std::vector<KronBuf> kb;
  for (size_t i0 = 0; i0 < refs.size();) {
    const auto nb = next_batch(i0, false, nk1);
    const size_t i1 = nb.first;
    st = ensure_kws(cx, nb.second);
    if (st != RBMC_OK) return st;
    st = carve_batch(i0, i1, false, nk1, kb);
    if (st != RBMC_OK) return st;
    double tb = now_s();
    st = kron_det_batch(cx, ms, refs, i0, i1, kb, L, lidx, diag_out, s, rep);
    if (st != RBMC_OK) return st;
    t_fac += now_s() - tb;
    if (nk1 > 0) {
      tb = now_s();
      st = kron_corr_batch(cx, ms, h1, nk1, x1, refs, i0, i1, kb, L, lidx, diag_out, mixed,
                           false, 1.0 / nk1, 0, s);
      if (st != RBMC_OK) return st;
      t_cor += now_s() - tb;
    }
    i0 = i1;
  }
  // Alg. 2 separator nodes: their variance from the samples (with several
  // passes zero here, so that the deterministic copy holds zero, then added
  // per pass)
  if (npass > 1)
    sep_variance(ms, h1, 0, nullptr, 0.0, 0, diag_out, s);
  else
    sep_variance(ms, h1, nk1, nk1 > 0 ? x1 : nullptr, nk1 > 0 ? 1.0 / nk1 : 0.0, 0, diag_out, s);
  HIPCHK(hipGetLastError());
  if (npass > 1) {
    for (size_t j = 0; j < ms.size(); ++j)
      HIPCHK(hipMemcpyAsync(ddet[j], diag_out[j], (size_t)ms[j]->plan.n * 8,
                            hipMemcpyDeviceToDevice, s));
    for (int c = 0; c < npass; ++c) {
      const int k0 = c * chunk, kn = std::min(chunk, nk_total - k0);
      const double* xc = x1;
      HostCols hc = h1;
      if (c > 0) {
        st = draw(k0, kn, &xc, &hc);
        if (st != RBMC_OK) return st;
      }
      const double tb = now_s();
      for (size_t i0 = 0; i0 < refs.size();) {
        const auto nb = next_batch(i0, true, kn);
        const size_t i1 = nb.first;
        st = ensure_kws(cx, nb.second);
        if (st != RBMC_OK) return st;
        st = carve_batch(i0, i1, true, kn, kb);
        if (st != RBMC_OK) return st;
        st = kron_corr_batch(cx, ms, hc, kn, xc, refs, i0, i1, kb, L, lidx, diag_out, mixed,
                             true, 1.0 / nk_total, c > 0 ? 1 : 0, s);
        if (st != RBMC_OK) return st;
        i0 = i1;
      }
      sep_variance(ms, hc, kn, xc, 1.0 / nk_total, 1, diag_out, s);
      HIPCHK(hipGetLastError());
      t_cor += now_s() - tb;
    }
  }
  st = combine_traces(cx, L, ms, nk_total, o, trace_out, rep);
  if (st != RBMC_OK) return st;
  if (rep && npass > 1) {  // plug-in error from the Monte Carlo share of each node
    size_t n_total = 0;
    double share = 0.0;
    for (size_t j = 0; j < ms.size(); ++j) {
      const size_t n = ms[j]->plan.n;
      n_total += n;
      const int nbk = mc_share_blocks(n);
      launch_mc_share(diag_out[j], ddet[j], n, cx->epart, s);
      std::vector<double> hp(nbk);
      HIPCHK(hipMemcpyAsync(hp.data(), cx->epart, nbk * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (double v : hp) share += v;
    }
    rep->err_estimate = std::sqrt(2.0 / M_PI) * std::sqrt(2.0 / nk_total) * share / n_total;
  }
  if (rep) {
    rep->t_sample = t_smp;
    rep->t_factor = t_fac;
    rep->t_select = 0.0;
    rep->t_correct = t_cor;
    rep->pcg_it_max = it_max;
    rep->pcg_it_mean = nk_total > 0 && sampler ? it_sum / nk_total : 0.0;
    rep->max_rel_residual = res_max;
    int64_t bytes = cx->ws.bytes + cx->epool.bytes + cx->kws.bytes + cx->kbank.bytes;
    for (rbmc_model* m : ms)
      bytes += m->pool.bytes + m->work_bj.bytes + m->work_sub.bytes + m->kpool.bytes +
               m->spool.bytes;
    rep->peak_bytes = bytes;
  }
  return st_s;
}

// RBMC_SEL_AUTO: the method with fewer dense flops for the set (Gauss-Jordan
// inversions of order n cost ~n^3; the block-tridiagonal method inverts one
// block per step of the two sweeps and per core step, the Kronecker method one
// spatial block per region and the capacitance matrix per subdomain, plus the
// product Z Y).
int resolve_method(const rbmc_est_opts* o, const std::vector<rbmc_model*>& ms) {
  if (o->method == RBMC_SEL_BLOCKTRI || o->method == RBMC_SEL_KRON) return o->method;
  double fb = 0.0, fk = 0.0;
  for (const rbmc_model* m : ms) {
    const Plan& P = m->plan;
    const double frac = P.n > 0 ? (double)m->n_obs / P.n : 0.0;
    std::vector<char> seen(P.regions.size(), 0);
    for (const Chain& c : P.sub) {
      const double nb = P.regions[c.region].nb();
      const int lc0 = c.ct0 - c.t0, lc1 = lc0 + c.cT - 1;
      fb += (double)(lc1 + (c.T - 1 - lc0) + c.cT) * nb * nb * nb;
      const double no = frac * c.T * nb;
      fk += no * no * no + 2.0 * nb * no * no;
      if (!seen[c.region]) {
        seen[c.region] = 1;
        fk += nb * nb * nb;
      }
    }
  }
  return fk < fb ? RBMC_SEL_KRON : RBMC_SEL_BLOCKTRI;
}

// Validate a set of models for one call.
rbmc_status check_models(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms) {
  for (rbmc_model* m : ms) {
    if (!m) return fail(RBMC_E_ARG, "model is NULL");
    if (m->ctx != cx) return fail(RBMC_E_ARG, "models must belong to the same context");
  }
  // a model's panels and factors are per model: it may appear only once
  std::vector<rbmc_model*> sorted(ms);
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(RBMC_E_ARG, "a model appears twice in one batched call");
  return RBMC_OK;
}

// Full path over a set: sample (caller's stream) || factor + core steps (side
// stream), then corrections.  z_ptrs: per model (n + n_obs) x n_k.
rbmc_status estimate_full(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms,
                          const rbmc_est_opts* opts, const std::vector<const double*>& z_ptrs,
                          const std::vector<double*>& diag_out,
                          const std::vector<double*>& trace_out, rbmc_report* rep,
                          bool device_z = false, uint64_t seed = 0) {
  const int nk = opts->n_samples;
  if (resolve_method(opts, ms) == RBMC_SEL_KRON) {
    // passes of `chunk` samples: z columns [k0, k0 + kn) of every model
    // (given, or drawn from seed + model index on the device), sampled on the
    // caller's stream
    const int chunk = (opts->sample_chunk > 0 && opts->sample_chunk < nk) ? opts->sample_chunk
                                                                          : std::max(nk, 1);
    if (!cols_fit(ms.size(), chunk))
      return fail(RBMC_E_ARG, "n_models * (samples per pass) exceeds 65535 columns");
    HostCols hpass;
    KronSampler smp = [&](int k0, int kn, const double** x, HostCols* hc,
                          rbmc_report* r) -> rbmc_status {
      *hc = make_cols(ms, kn);
      const bool cat = device_z || ms.size() > 1;
      rbmc_status e = ensure_ws(cx, ms, *hc, cat);
      if (e != RBMC_OK) return e;
      const double* zb = nullptr;
      if (cat) {
        for (size_t j = 0; j < ms.size(); ++j) {
          const size_t nz = (size_t)(ms[j]->plan.n + ms[j]->n_obs);
          if (device_z)
            launch_normals(seed + j, (size_t)k0 * nz, (size_t)kn * nz, cx->zcat + hc->zbase[j],
                           cx->stream);
          else
            HIPCHK(hipMemcpyAsync(cx->zcat + hc->zbase[j], z_ptrs[j] + (size_t)k0 * nz,
                                  (size_t)kn * nz * 8, hipMemcpyDeviceToDevice, cx->stream));
        }
        HIPCHK(hipGetLastError());
        zb = cx->zcat;
      } else {
        zb = z_ptrs[0] + (size_t)k0 * (ms[0]->plan.n + ms[0]->n_obs);
      }
      rbmc_est_opts oc = *opts;
      oc.n_samples = kn;
      e = sample_set(cx, ms, *hc, &oc, zb, cx->x, r, cx->stream);
      *x = cx->x;
      return e;
    };
    rbmc_status st = estimate_set_kron(cx, ms, opts, nk, chunk, smp, nullptr, nullptr, diag_out,
                                       trace_out, rep);
    (void)hpass;
    return st;
  }
  if (device_z) return fail(RBMC_E_UNSUPPORTED, "device normals need RBMC_SEL_KRON");
  if (!cols_fit(ms.size(), nk))
    return fail(RBMC_E_ARG, "n_models * n_samples exceeds 65535 columns per call");
  const HostCols h = make_cols(ms, nk);
  const bool single = ms.size() == 1;
  rbmc_status st = ensure_ws(cx, ms, h, !single && nk > 0);
  if (st != RBMC_OK) return st;
  const double* zb = nullptr;
  if (nk > 0) {
    if (single) {
      zb = z_ptrs[0];
    } else {
      for (size_t j = 0; j < ms.size(); ++j)
        HIPCHK(hipMemcpyAsync(cx->zcat + h.zbase[j], z_ptrs[j],
                              (size_t)(ms[j]->plan.n + ms[j]->n_obs) * nk * 8,
                              hipMemcpyDeviceToDevice, cx->stream));
      zb = cx->zcat;
    }
  }
  rbmc_status st1 = RBMC_OK;
  std::function<rbmc_status()> sampler;
  if (nk > 0 && cx->overlap)
    sampler = [&]() -> rbmc_status {
      st1 = sample_set(cx, ms, h, opts, zb, cx->x, rep, cx->work);
      return st1;
    };
  if (nk > 0 && !cx->overlap) {  // sample first, then everything else, on one stream
    st1 = sample_set(cx, ms, h, opts, zb, cx->x, rep, cx->stream);
    if (st1 < 0) return st1;
  }
  st = estimate_set(cx, ms, h, opts, cx->x, diag_out, trace_out, rep, sampler);
  if (st < 0) return st;
  return st1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free operator application (rbmc_apply_op_noalloc).  Its column
// tables and the model view live in `scratch`, a file-scope device array of
// kScratchBytes per device that the library never allocates or frees.  Host
// code never uses the array's name as an address: rbmc_ctx_create resolves
// the address on each device once (hipGetSymbolAddress, with that device
// current) and the entry point passes that address to its kernels.  Every
// call on a device shares the device's array: calls that overlap on one
// device race.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)2 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device; nullptr until resolved

// column c of one model: n entries at c n, operator input at c (n + n_obs);
// block 0 also copies the model view (words 8-byte units)
__global__ void k_fill_cols(int64_t* __restrict__ off, int64_t* __restrict__ in_off,
                            int* __restrict__ len, int* __restrict__ model, int ncols, int n,
                            int n_obs, const uint64_t* __restrict__ view_src,
                            uint64_t* __restrict__ view_dst, int words) {
  if (blockIdx.x == 0 && (int)threadIdx.x < words) view_dst[threadIdx.x] = view_src[threadIdx.x];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  off[c] = (int64_t)c * n;
  in_off[c] = (int64_t)c * (n + n_obs);
  len[c] = n;
  model[c] = 0;
}

// Resolve (once per device) the device address of `scratch`; `device` must
// be current.  Empty launches on stream s then make the runtime load the
// device code the allocation-free entry point runs (this file's and the
// operator kernels'; each source file is its own code object, loaded on the
// first launch of one of its kernels) now, not inside a later call.
rbmc_status scratch_resolve(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device]) return RBMC_OK;
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  k_fill_cols<<<1, 64, 0, s>>>(nullptr, nullptr, nullptr, nullptr, 0, 0, 0, nullptr, nullptr, 0);
  load_stencil_module(s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  g_scratch_ptr[device] = ptr;
  return RBMC_OK;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

// Layout of the column tables in the scratch block: the model view, then
// off, in_off (int64) and len, model (int32) of ncols columns.
struct ScratchCols {
  DevModel* dm;
  int64_t *off, *in_off;
  int *len, *model;
};
constexpr size_t kScratchView = 512;  // bytes reserved for the model view
size_t scratch_cols_bytes(int ncols) { return kScratchView + (size_t)ncols * 24; }
ScratchCols scratch_layout(void* base, int ncols) {
  char* p = (char*)base;
  ScratchCols c;
  c.dm = (DevModel*)p;
  c.off = (int64_t*)(p + kScratchView);
  c.in_off = c.off + ncols;
  c.len = (int*)(c.in_off + ncols);
  c.model = c.len + ncols;
  return c;
}
static_assert(sizeof(DevModel) <= kScratchView, "model view exceeds its scratch slot");
}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
namespace {
// workload signature of an autotuning: device, options, every model's grid
// and decomposition
std::string tune_signature(rbmc_ctx* cx, const std::vector<rbmc_model*>& ms,
                           const rbmc_est_opts* o) {
  hipDeviceProp_t prop;
  std::ostringstream os;
  if (hipGetDeviceProperties(&prop, cx->device) == hipSuccess) os << prop.gcnArchName;
  os << "|nk" << o->n_samples << " prec" << o->precision << " pc" << o->precond << " g"
     << o->grad_mask;
  for (const rbmc_model* m : ms) {
    const rbmc_decomp_desc& d = m->dc;
    os << "|" << m->plan.mx << "x" << m->plan.my << "x" << m->plan.T << " " << d.n_tslabs << ","
       << d.n_tiles_x << "," << d.n_tiles_y << "," << d.overlap_hops << " " << d.pc_tslabs << ","
       << d.pc_tiles_x << "," << d.pc_tiles_y;
  }
  return os.str();
}

std::string tune_key(const std::string& sig) {  // FNV-1a, 64 bit
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : sig) {
    h ^= c;
    h *= 1099511628211ull;
  }
  char buf[17];
  std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return buf;
}

// cache line: <key> <small_k> <small_tiles> <wide_from> <best_ms> <signature>
bool tune_cache_lookup(const char* path, const std::string& key, Tune* t, double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    Tune v;
    double b = 0.0;
    if (!(is >> k >> v.small_k >> v.small_tiles >> v.wide_from >> b) || k != key) continue;
    if (v.small_k < 0 || v.small_tiles < 0 || v.wide_from < kSweepWideFrom) continue;
    *t = v;
    *ms = b;
    return true;
  }
  return false;
}
}  // namespace

extern "C" {

const char* rbmc_last_error(void) { return g_err.c_str(); }

rbmc_status rbmc_ctx_profile(rbmc_ctx* ctx, int enable) {
  if (!ctx) return fail(RBMC_E_ARG, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->clear();
  ctx->prof = enable != 0;
  return RBMC_OK;
}

rbmc_status rbmc_ctx_profile_read(rbmc_ctx* ctx, int family, rbmc_kernel_stats* out) {
  if (!ctx || !out) return fail(RBMC_E_ARG, "NULL argument");
  if (family < 0 || family >= RBMC_KF_COUNT) return fail(RBMC_E_ARG, "unknown kernel family");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (hipStream_t q : {ctx->side, ctx->side2, ctx->work})
    if (q) HIPCHK(hipStreamSynchronize(q));
  std::memset(out, 0, sizeof(*out));
  for (const ProfRec& r : ctx->recs) {
    if (r.family != family) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    out->launches += 1;
    out->total_ms += ms;
    out->alg_flops += r.flops;
    out->alg_bytes += r.bytes;
  }
  return RBMC_OK;
}

rbmc_status rbmc_ctx_create(int device, void* hip_stream, rbmc_ctx** out) {
  if (!out) return fail(RBMC_E_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(RBMC_E_ARG, "no such device");
  HIPCHK(hipSetDevice(device));
  {  // the allocation-free entry point's scratch block on this device
    rbmc_status st = scratch_resolve(device, (hipStream_t)hip_stream);
    if (st != RBMC_OK) return st;
  }
  rbmc_ctx* c = new rbmc_ctx;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (const char* e = std::getenv("RBMC_OVERLAP")) c->overlap = std::atoi(e) != 0;
  if (const char* e = std::getenv("RBMC_LAUNCH_THREADS")) c->launch_threads = std::atoi(e) > 1;
  if (const char* e = std::getenv("RBMC_RESERVE_CUS")) c->reserve_cus = std::atoi(e);
  if (const char* e = std::getenv("RBMC_KRON_BATCH_BYTES"))
    c->kron_batch_cap = (size_t)std::strtoull(e, nullptr, 10);
  *out = c;
  return RBMC_OK;
}

void rbmc_ctx_destroy(rbmc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  delete ctx;
}

rbmc_status rbmc_plan_query(const rbmc_model_desc* desc, const rbmc_decomp_desc* decomp,
                            int32_t p, int32_t* label_out, uint8_t* state_out) {
  if (!desc || !decomp) return fail(RBMC_E_ARG, "desc/decomp is NULL");
  Plan plan;
  std::string e = make_plan(*desc, *decomp, plan);
  if (!e.empty()) return fail(RBMC_E_ARG, e);
  if (label_out) plan_labels(plan, label_out);
  if (state_out) {
    if (p < 0 || p >= (int)plan.sub.size()) return fail(RBMC_E_ARG, "core index out of range");
    plan_state(plan, p, state_out);
  }
  return RBMC_OK;
}

rbmc_status rbmc_model_create(rbmc_ctx* ctx, const rbmc_model_desc* desc,
                              const rbmc_decomp_desc* decomp, rbmc_model** out) {
  if (!ctx || !desc || !decomp || !out) return fail(RBMC_E_ARG, "NULL argument");
  *out = nullptr;
  if (!(desc->h > 0.0) || !std::isfinite(desc->h)) return fail(RBMC_E_ARG, "h must be > 0");
  if (!theta_ok(desc->log_kappa, desc->log_tau, desc->rho, desc->log_sigma))
    return fail(RBMC_E_ARG, "theta must be finite with |rho| < 1");
  if (!desc->obs_mask) return fail(RBMC_E_ARG, "obs_mask is NULL");
  Plan plan;
  std::string e = make_plan(*desc, *decomp, plan);
  if (!e.empty()) return fail(RBMC_E_ARG, e);
  HIPCHK(hipSetDevice(ctx->device));
  rbmc_model* m = new rbmc_model;
  m->ctx = ctx;
  m->desc = *desc;
  m->dc = *decomp;
  m->plan = std::move(plan);
  const Plan& P = m->plan;
  m->mask.assign(desc->obs_mask, desc->obs_mask + P.n);
  for (uint8_t v : m->mask) m->n_obs += v ? 1 : 0;
  m->desc.obs_mask = m->mask.data();
  make_coefs(P.mx, P.my, P.T, desc->h, desc->log_kappa, desc->log_tau, desc->rho,
             desc->log_sigma, m->co);
  auto cleanup = [&](rbmc_status st) {
    m->work_bj.release();
    m->work_sub.release();
    m->kpool.release();
    m->spool.release();
    m->pool.release();
    delete m;
    return st;
  };
#define MCHK(expr)                                                                  \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return cleanup(fail(e_ == hipErrorOutOfMemory ? RBMC_E_OOM : RBMC_E_DEVICE,   \
                          std::string(#expr) + ": " + hipGetErrorString(e_)));      \
  } while (0)
  MCHK(m->pool.alloc((void**)&m->d_qs, m->co.qs.size() * 8));
  MCHK(m->pool.alloc((void**)&m->d_kk, m->co.kk.size() * 8));
  MCHK(m->pool.alloc((void**)&m->d_fs, m->co.fs.size() * 8));
  MCHK(m->pool.alloc((void**)&m->d_qd, (size_t)P.T * 8));
  MCHK(m->pool.alloc((void**)&m->d_dqd, (size_t)P.T * 8));
  MCHK(m->pool.alloc((void**)&m->d_ld, (size_t)P.T * 8));
  MCHK(m->pool.alloc((void**)&m->d_dvec, (size_t)P.n * 8));
  MCHK(m->pool.alloc((void**)&m->d_obs_rank, (size_t)P.n * 4));
  const size_t nwords = ((size_t)P.n + 31) / 32;
  MCHK(m->pool.alloc((void**)&m->d_obs_bits, nwords * 4));
  MCHK(m->pool.alloc((void**)&m->d_obs_wrank, nwords * 4));
  MCHK(m->pool.alloc((void**)&m->d_dm, sizeof(DevModel)));
  {
    std::vector<int> rank(P.n, -1);
    std::vector<uint32_t> bits(nwords, 0u);
    std::vector<int> wrank(nwords, 0);
    int r = 0;
    for (int i = 0; i < P.n; ++i) {
      if ((i & 31) == 0) wrank[i >> 5] = r;
      if (m->mask[i]) {
        bits[i >> 5] |= 1u << (i & 31);
        rank[i] = r++;
      }
    }
    MCHK(hipMemcpy(m->d_obs_rank, rank.data(), (size_t)P.n * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(m->d_obs_bits, bits.data(), nwords * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(m->d_obs_wrank, wrank.data(), nwords * 4, hipMemcpyHostToDevice));
  }
  if (!P.sep_nodes.empty()) {
    MCHK(m->pool.alloc((void**)&m->d_sep, P.sep_nodes.size() * 4));
    MCHK(hipMemcpy(m->d_sep, P.sep_nodes.data(), P.sep_nodes.size() * 4, hipMemcpyHostToDevice));
  }
  DevModel& dm = m->dm;
  dm.mx = P.mx;
  dm.my = P.my;
  dm.T = P.T;
  dm.ns = P.ns;
  dm.n = P.n;
  dm.n_obs = m->n_obs;
  dm.qs = m->d_qs;
  dm.kk = m->d_kk;
  dm.fs = m->d_fs;
  dm.qd = m->d_qd;
  dm.dqd = m->d_dqd;
  dm.ld = m->d_ld;
  dm.dvec = m->d_dvec;
  dm.obs_rank = m->d_obs_rank;
  dm.obs_bits = m->d_obs_bits;
  dm.obs_wrank = m->d_obs_wrank;
  // regions
  for (const Region& g : P.regions) {
    RegionDev rd{};
    rd.nb = g.nb();
    rd.np = pad_to(rd.nb);
    int *nodes = nullptr, *nbr = nullptr;
    uint8_t* ib = nullptr;
    MCHK(m->pool.alloc((void**)&nodes, g.nodes.size() * 4));
    MCHK(m->pool.alloc((void**)&nbr, g.nbr.size() * 4));
    MCHK(m->pool.alloc((void**)&ib, g.in_box.size()));
    MCHK(hipMemcpy(nodes, g.nodes.data(), g.nodes.size() * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(nbr, g.nbr.data(), g.nbr.size() * 4, hipMemcpyHostToDevice));
    MCHK(hipMemcpy(ib, g.in_box.data(), g.in_box.size(), hipMemcpyHostToDevice));
    rd.nodes = nodes;
    rd.nbr = nbr;
    rd.in_box = ib;
    m->regions.push_back(rd);
  }
  MCHK(m->pool.alloc((void**)&m->d_regions, m->regions.size() * sizeof(RegionDev)));
  MCHK(hipMemcpy(m->d_regions, m->regions.data(), m->regions.size() * sizeof(RegionDev),
                 hipMemcpyHostToDevice));
  MCHK(m->pool.alloc((void**)&m->d_info, (P.bj.size() + P.sub.size()) * 4));
  {
    // the chain sets, the Kronecker data and the spectral data are allocated
    // by the first call that uses them
    rbmc_status st = upload_coefs(m);
    if (st != RBMC_OK) return cleanup(st);
  }
#undef MCHK
  *out = m;
  return RBMC_OK;
}

void rbmc_model_destroy(rbmc_model* m) {
  if (!m) return;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  for (hipStream_t q : {m->ctx->side, m->ctx->side2, m->ctx->work})
    if (q) (void)hipStreamSynchronize(q);
  m->work_bj.release();
  m->work_sub.release();
  m->kpool.release();
  m->spool.release();
  m->lwork.release();
  m->pool.release();
  delete m;
}

rbmc_status rbmc_model_set_theta(rbmc_model* m, double log_kappa, double log_tau, double rho,
                                 double log_sigma) {
  if (!m) return fail(RBMC_E_ARG, "model is NULL");
  if (!theta_ok(log_kappa, log_tau, rho, log_sigma))
    return fail(RBMC_E_ARG, "theta must be finite with |rho| < 1");
  m->desc.log_kappa = log_kappa;
  m->desc.log_tau = log_tau;
  m->desc.rho = rho;
  m->desc.log_sigma = log_sigma;
  make_coefs(m->plan.mx, m->plan.my, m->plan.T, m->desc.h, log_kappa, log_tau, rho, log_sigma,
             m->co);
  return upload_coefs(m);
}

rbmc_status rbmc_apply_op(rbmc_model* m, int op, const double* x, double* y, int32_t n_rhs) {
  if (!m || !x || !y) return fail(RBMC_E_ARG, "NULL argument");
  if (op < RBMC_OP_Q || op > RBMC_OP_F) return fail(RBMC_E_ARG, "unknown operator");
  if (n_rhs < 0) return fail(RBMC_E_ARG, "n_rhs must be >= 0");
  if (n_rhs == 0) return RBMC_OK;
  if (!cols_fit(1, n_rhs)) return fail(RBMC_E_ARG, "n_rhs exceeds 65535");
  HIPCHK(hipSetDevice(m->ctx->device));
  std::vector<rbmc_model*> ms{m};
  const HostCols h = make_cols(ms, n_rhs);
  rbmc_status st = ensure_ws(m->ctx, ms, h, false);
  if (st != RBMC_OK) return st;
  launch_apply_op(colset(m->ctx, h), op, x, y, m->ctx->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(m->ctx->stream));
  return RBMC_OK;
}

rbmc_status rbmc_apply_op_noalloc(rbmc_model* m, int op, const double* x, double* y,
                                  int32_t n_rhs) {
  if (!m || !x || !y) return fail(RBMC_E_ARG, "NULL argument");
  if (op < RBMC_OP_Q || op > RBMC_OP_F) return fail(RBMC_E_ARG, "unknown operator");
  if (n_rhs < 0) return fail(RBMC_E_ARG, "n_rhs must be >= 0");
  if (n_rhs == 0) return RBMC_OK;
  if (n_rhs > (int32_t)kMaxCols || scratch_cols_bytes(n_rhs) > kScratchBytes)
    return fail(RBMC_E_ARG, "n_rhs exceeds 65535 columns (the scratch block's limit)");
  const int dev = m->ctx->device;
  HIPCHK(hipSetDevice(dev));
  void* base = scratch_of(dev);
  if (!base) return fail(RBMC_E_DEVICE, "scratch block not resolved on this device");
  hipStream_t s = m->ctx->stream;
  const ScratchCols t = scratch_layout(base, n_rhs);
  static_assert(sizeof(DevModel) % 8 == 0 && sizeof(DevModel) / 8 <= 256, "model view words");
  k_fill_cols<<<(n_rhs + 255) / 256, 256, 0, s>>>(
      t.off, t.in_off, t.len, t.model, n_rhs, m->plan.n, m->n_obs, (const uint64_t*)m->d_dm,
      (uint64_t*)t.dm, (int)(sizeof(DevModel) / 8));
  ColSet cs{};
  cs.ncols = n_rhs;
  cs.max_len = m->plan.n;
  cs.max_tiles = stencil_tiles(m->plan.mx, m->plan.my);
  cs.max_ns = m->plan.ns;
  cs.max_T = m->plan.T;
  cs.off = t.off;
  cs.in_off = t.in_off;
  cs.len = t.len;
  cs.model = t.model;
  cs.dms = t.dm;
  launch_apply_op(cs, op, x, y, s);
  HIPCHK(hipGetLastError());
  return RBMC_OK;
}

rbmc_status rbmc_sample(rbmc_model* m, const rbmc_est_opts* opts, const double* z, double* x,
                        rbmc_report* rep) {
  init_report(rep);
  if (!m || !z || !x) return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (opts->n_samples == 0) return RBMC_OK;
  if (!cols_fit(1, opts->n_samples)) return fail(RBMC_E_ARG, "n_samples exceeds 65535");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  std::vector<rbmc_model*> ms{m};
  const HostCols h = make_cols(ms, opts->n_samples);
  st = ensure_ws(m->ctx, ms, h, false);
  if (st != RBMC_OK) return st;
  st = sample_set(m->ctx, ms, h, opts, z, x, rep, m->ctx->stream);
  if (rep) {
    rep->t_total = now_s() - t0;
    rep->peak_bytes = m->ctx->ws.bytes + m->pool.bytes + m->work_bj.bytes + m->spool.bytes;
  }
  return st;
}

rbmc_status rbmc_solve(rbmc_model* m, const rbmc_est_opts* opts, const double* b, double* x,
                       rbmc_report* rep) {
  init_report(rep);
  if (!m || !b || !x) return fail(RBMC_E_ARG, "NULL argument");
  if (b == x) return fail(RBMC_E_ARG, "b and x must be distinct buffers");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (opts->n_samples == 0) return RBMC_OK;
  if (!cols_fit(1, opts->n_samples)) return fail(RBMC_E_ARG, "n_samples exceeds 65535");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  std::vector<rbmc_model*> ms{m};
  const HostCols h = make_cols(ms, opts->n_samples);
  st = ensure_ws(m->ctx, ms, h, false);
  if (st != RBMC_OK) return st;
  st = sample_set(m->ctx, ms, h, opts, nullptr, x, rep, m->ctx->stream, {}, b);
  if (rep) {
    rep->t_total = now_s() - t0;
    rep->peak_bytes = m->ctx->ws.bytes + m->pool.bytes + m->work_bj.bytes + m->spool.bytes;
  }
  return st;
}

rbmc_status rbmc_probe_overlap(rbmc_model* m, const rbmc_est_opts* opts, double eps,
                               int32_t* lags, double* corr_time, double* corr_space) {
  if (!m || !opts || !lags) return fail(RBMC_E_ARG, "NULL argument");
  if (!(eps > 0.0 && eps < 1.0)) return fail(RBMC_E_ARG, "eps must lie in (0, 1)");
  const Plan& P = m->plan;
  const int ns = P.ns, T = P.T, mx = P.mx, my = P.my;
  const int tc = T / 2, cx = mx / 2, cy = my / 2;
  const size_t n = (size_t)P.n, c = (size_t)tc * ns + (size_t)cy * mx + cx;
  HIPCHK(hipSetDevice(m->ctx->device));
  double* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, 2 * n * sizeof(double)));
  double* b = d;
  double* y = d + n;
  std::vector<double> hy(n);
  rbmc_est_opts o = *opts;
  o.n_samples = 1;
  o.sample_chunk = 0;
  rbmc_status st = RBMC_OK;
  const double one = 1.0;
  hipError_t e = hipMemsetAsync(b, 0, n * sizeof(double), m->ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + c, &one, sizeof(double), hipMemcpyHostToDevice, m->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->ctx->stream);
  if (e == hipSuccess) {
    st = rbmc_solve(m, &o, b, y, nullptr);
    if (st >= 0) e = hipMemcpy(hy.data(), y, n * sizeof(double), hipMemcpyDeviceToHost);
  }
  (void)hipFree(d);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? RBMC_E_OOM : RBMC_E_DEVICE, hipGetErrorString(e));
  if (st < 0) return st;
  const double yc = hy[c];
  if (!(yc > 0.0)) return fail(RBMC_E_NOT_SPD, "non-positive variance at the probe node");
  // time: the centre's spatial node at every step; space: every node of the
  // centre's step, by L1 grid distance.  lag = the smallest distance from
  // which on every ratio |y_j| / y_c is at most eps
  const size_t sc = (size_t)cy * mx + cx;
  int lag_t = 1;
  for (int t = 0; t < T; ++t) {
    const double r = hy[(size_t)t * ns + sc] / yc;
    if (corr_time) corr_time[t] = r;
    if (std::fabs(r) > eps) lag_t = std::max(lag_t, std::abs(t - tc) + 1);
  }
  int lag_s = 1;
  for (int iy = 0; iy < my; ++iy)
    for (int ix = 0; ix < mx; ++ix) {
      const size_t s = (size_t)iy * mx + ix;
      const double r = hy[(size_t)tc * ns + s] / yc;
      if (corr_space) corr_space[s] = r;
      if (std::fabs(r) > eps) lag_s = std::max(lag_s, std::abs(ix - cx) + std::abs(iy - cy) + 1);
    }
  lags[0] = lag_t;
  lags[1] = lag_s;
  lags[2] = std::max(lag_t, (lag_s + 1) / 2);
  return st;
}

rbmc_status rbmc_posterior_mean(rbmc_model* m, const rbmc_est_opts* opts, const double* y,
                                int32_t n_beta, const double* a_beta, const double* q_beta,
                                double* mu_u, double* mu_beta, double* var_beta,
                                double* var_u_add, rbmc_report* rep) {
  init_report(rep);
  if (!m || !opts || !mu_u) return fail(RBMC_E_ARG, "NULL argument");
  if (n_beta < 0 || n_beta > RBMC_MAX_FIXED_EFFECTS)
    return fail(RBMC_E_ARG, "n_beta must lie in [0, RBMC_MAX_FIXED_EFFECTS]");
  const int n_obs = m->n_obs;
  if (n_obs > 0 && !y) return fail(RBMC_E_ARG, "y is NULL");
  if (n_beta > 0 && ((n_obs > 0 && !a_beta) || !q_beta || !mu_beta))
    return fail(RBMC_E_ARG, "a_beta, q_beta or mu_beta is NULL");
  for (int j = 0; j < n_beta; ++j)
    if (!(std::isfinite(q_beta[j]) && q_beta[j] > 0.0))
      return fail(RBMC_E_ARG, "q_beta entries must be finite and positive");
  const int n = m->plan.n, nc = n_beta + 1, np = n_beta * nc;
  const double tau_y = m->co.dobs;
  HIPCHK(hipSetDevice(m->ctx->device));
  const double t0 = now_s();
  hipStream_t s = m->ctx->stream;
  // B and W (n x nc each), the Gram partials, G = Q_betau [w W],
  // H = A_beta^T [y A_beta], the prior precisions and the Schur results
  const int nblk = std::max(mean_gram_blocks(n), mean_gram_blocks(n_obs));
  const size_t nsol = 1 + (size_t)n_beta + (size_t)n_beta * n_beta;
  const size_t words = 2 * (size_t)n * nc + (size_t)nblk * np + 2 * (size_t)np + n_beta + nsol;
  double* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, words * sizeof(double)));
  double* B = d;
  double* W = B + (size_t)n * nc;
  double* part = W + (size_t)n * nc;
  double* Gm = part + (size_t)nblk * np;
  double* Hm = Gm + np;
  double* q = Hm + np;
  double* sol = q + n_beta;
  std::vector<double> hsol(nsol, 0.0);
  rbmc_status st = RBMC_OK;
  hipError_t e = hipSuccess;
  launch_mean_rhs(n, n_obs, m->d_obs_rank, tau_y, y, a_beta, n_beta, B, (size_t)n, s);
  e = hipGetLastError();
  if (e == hipSuccess) {
    rbmc_est_opts o = *opts;
    o.n_samples = nc;
    o.sample_chunk = 0;
    st = rbmc_solve(m, &o, B, W, rep);
  }
  if (e == hipSuccess && st >= 0 && n_beta > 0) {
    // Q_betau [w W]: the covariate columns of B are Q_ubeta's
    launch_mean_gram(n, n_beta, B + n, (size_t)n, nc, W, W + n, (size_t)n, part, Gm, s);
    launch_mean_gram(n_obs, n_beta, a_beta, (size_t)n_obs, nc, y, a_beta, (size_t)n_obs, part,
                     Hm, s);
    e = hipMemcpyAsync(q, q_beta, (size_t)n_beta * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      launch_mean_schur(n_beta, Gm, Hm, q, tau_y, sol, s);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess && st >= 0) {
    launch_mean_combine(n, n_beta, W, (size_t)n, sol, mu_u, var_u_add, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess && st >= 0 && n_beta > 0)
    e = hipMemcpyAsync(hsol.data(), sol, nsol * sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  (void)hipFree(d);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? RBMC_E_OOM : RBMC_E_DEVICE, hipGetErrorString(e));
  if (st < 0) return st;
  if (n_beta > 0) {
    if (hsol[0] != 0.0)
      return fail(RBMC_E_NOT_SPD, "Schur complement of the fixed effects not positive definite "
                                  "at pivot " + std::to_string((int)hsol[0] - 1));
    for (int j = 0; j < n_beta; ++j) mu_beta[j] = hsol[1 + j];
    if (var_beta)
      for (int j = 0; j < n_beta * n_beta; ++j) var_beta[j] = hsol[1 + n_beta + j];
  }
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_grad_log_posterior(rbmc_model* m, const rbmc_est_opts* opts, const double* y,
                                    const double* x, uint64_t seed, double* grad_out,
                                    double* terms_out, double* mu_out, rbmc_report* rep) {
  init_report(rep);
  if (!m || !opts || !grad_out) return fail(RBMC_E_ARG, "NULL argument");
  const int n_obs = m->n_obs;
  if (n_obs > 0 && !y) return fail(RBMC_E_ARG, "y is NULL");
  const Plan& P = m->plan;
  const int n = P.n;
  HIPCHK(hipSetDevice(m->ctx->device));
  const double t0 = now_s();
  hipStream_t s = m->ctx->stream;
  // mu (unless the caller's buffer), the estimator's diagonal, d_j Q mu
  // (4 columns), y on the grid, Gram partials and six sums
  const int nblk = std::max(mean_gram_blocks(n), mean_gram_blocks(n_obs));
  const size_t words = 7 * (size_t)n + (size_t)nblk * 4 + 8;
  double* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, words * sizeof(double)));
  double* mu = mu_out ? mu_out : d;
  double* diag = d + n;
  double* dq = diag + n;
  double* yg = dq + 4 * (size_t)n;
  double* part = yg + n;
  double* sums = part + (size_t)nblk * 4;
  double hs[6] = {0, 0, 0, 0, 0, 0};
  double tr[4] = {0, 0, 0, 0};
  rbmc_report rm{}, re{};
  hipError_t e = hipSuccess;
  rbmc_status st_w = RBMC_OK;  // the larger warning of the two calls
  // mu = Q^-1 A_u^T Q_y y (eq:mean:1)
  rbmc_status st = rbmc_posterior_mean(m, opts, y, 0, nullptr, nullptr, mu, nullptr, nullptr,
                                       nullptr, &rm);
  if (st > st_w) st_w = st;
  // tr(Q^-1 d_j Q) by the estimator (eq:hyperpar:4)
  if (st >= 0) {
    rbmc_est_opts eo = *opts;
    eo.grad_mask = 0xF;
    if (x || opts->n_samples == 0)
      st = rbmc_estimate_from_samples(m, &eo, x, diag, tr, &re);
    else
      st = rbmc_estimate(m, &eo, nullptr, seed, diag, tr, &re);
    if (st > st_w) st_w = st;
  }
  // mu^T d_j Q mu, sum_o y_o mu_o (y scattered to the grid) and sum_o y_o^2
  for (int j = 0; st >= 0 && j < 4; ++j)
    st = rbmc_apply_op(m, RBMC_OP_DQ_LOGKAPPA + j, mu, dq + (size_t)j * n, 1);
  if (st >= 0) {
    launch_mean_gram(n, 1, mu, (size_t)n, 4, dq, dq + n, (size_t)n, part, sums, s);
    launch_mean_rhs(n, n_obs, m->d_obs_rank, 1.0, y, nullptr, 0, yg, (size_t)n, s);
    launch_mean_gram(n, 1, yg, (size_t)n, 1, mu, nullptr, (size_t)n, part, sums + 4, s);
    launch_mean_gram(n_obs, 1, y, (size_t)n_obs, 1, y, nullptr, (size_t)n_obs, part, sums + 5, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, s);
  }
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  (void)hipFree(d);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? RBMC_E_OOM : RBMC_E_DEVICE, hipGetErrorString(e));
  if (st < 0) return st;
  // prior log-determinant derivatives in closed form
  const double kappa2 = std::exp(2.0 * m->desc.log_kappa), h = m->desc.h, rho = m->desc.rho;
  const double kh2 = kappa2 * h * h;
  std::vector<double> lx(P.mx), ly(P.my);
  for (int a = 0; a < P.mx; ++a) lx[a] = 2.0 - 2.0 * std::cos(M_PI * a / P.mx);
  for (int b = 0; b < P.my; ++b) ly[b] = 2.0 - 2.0 * std::cos(M_PI * b / P.my);
  double sk = 0.0;
  for (int b = 0; b < P.my; ++b)
    for (int a = 0; a < P.mx; ++a) sk += 1.0 / (kh2 + lx[a] + ly[b]);
  const double prior[4] = {0.5 * P.T * 4.0 * kh2 * sk, 0.5 * (double)n,
                           (double)P.ns * (P.T - 1) * rho / (1.0 - rho * rho), 0.0};
  // ||r||^2 = sum y^2 - 2 sum y mu_obs + sum mu_obs^2, the last from
  // mu^T d_logsigma Q mu = -2 tau_y sum mu_obs^2
  const double tau_y = m->co.dobs;
  const double mu_obs2 = -hs[3] / (2.0 * tau_y);
  const double r2 = hs[5] - 2.0 * hs[4] + mu_obs2;
  for (int j = 0; j < 4; ++j) {
    const double t[5] = {j == 3 ? -(double)n_obs : 0.0, prior[j], -0.5 * tr[j],
                         j == 3 ? tau_y * r2 : 0.0, j < 3 ? -0.5 * hs[j] : 0.0};
    grad_out[j] = t[0] + t[1] + t[2] + t[3] + t[4];
    if (terms_out)
      for (int k = 0; k < 5; ++k) terms_out[j * 5 + k] = t[k];
  }
  if (rep) {
    *rep = re;
    rep->pcg_it_max = std::max(re.pcg_it_max, rm.pcg_it_max);
    rep->t_total = now_s() - t0;
  }
  return st_w;
}

rbmc_status rbmc_estimate_from_samples(rbmc_model* m, const rbmc_est_opts* opts, const double* x,
                                       double* diag_out, double* trace_out, rbmc_report* rep) {
  init_report(rep);
  if (!m || !diag_out) return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, false);
  if (st != RBMC_OK) return st;
  if (opts->n_samples > 0 && !x) return fail(RBMC_E_ARG, "x is NULL");
  if (opts->grad_mask && !trace_out) return fail(RBMC_E_ARG, "trace_out is NULL");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  std::vector<rbmc_model*> ms{m};
  const HostCols h = make_cols(ms, opts->n_samples);
  if (resolve_method(opts, ms) == RBMC_SEL_KRON)
    st = estimate_set_kron(m->ctx, ms, opts, opts->n_samples, std::max(opts->n_samples, 1), {}, x,
                           &h, {diag_out}, {trace_out}, rep);
  else
    st = estimate_set(m->ctx, ms, h, opts, x, {diag_out}, {trace_out}, rep, {});
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_estimate(rbmc_model* m, const rbmc_est_opts* opts, const double* z, uint64_t seed,
                          double* diag_out, double* trace_out, rbmc_report* rep) {
  init_report(rep);
  if (!m || !diag_out) return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (opts->grad_mask && !trace_out) return fail(RBMC_E_ARG, "trace_out is NULL");
  const bool device_z = opts->n_samples > 0 && !z;
  if (device_z && resolve_method(opts, {m}) != RBMC_SEL_KRON)
    return fail(RBMC_E_UNSUPPORTED, "z = NULL (device normals) needs the Kronecker method");
  if (opts->sample_chunk > 0 && opts->sample_chunk < opts->n_samples &&
      resolve_method(opts, {m}) != RBMC_SEL_KRON)
    return fail(RBMC_E_UNSUPPORTED, "sample_chunk < n_samples needs the Kronecker method");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  st = estimate_full(m->ctx, {m}, opts, {z}, {diag_out}, {trace_out}, rep, device_z, seed);
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_normals(rbmc_ctx* ctx, uint64_t seed, uint64_t offset, int64_t count,
                         double* out) {
  if (!ctx) return fail(RBMC_E_ARG, "ctx is NULL");
  if (count < 0) return fail(RBMC_E_ARG, "count must be >= 0");
  if (count == 0) return RBMC_OK;
  if (!out) return fail(RBMC_E_ARG, "out is NULL");
  HIPCHK(hipSetDevice(ctx->device));
  launch_normals(seed, offset, (size_t)count, out, ctx->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RBMC_OK;
}

rbmc_status rbmc_estimate_batched(rbmc_ctx* ctx, int32_t n_models, rbmc_model* const* models,
                                  const rbmc_est_opts* opts, const double* const* z,
                                  double* const* diag_out, double* const* trace_out,
                                  rbmc_report* rep) {
  init_report(rep);
  if (!ctx || n_models < 0 || (n_models > 0 && (!models || !diag_out)))
    return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (n_models == 0) return RBMC_OK;
  std::vector<rbmc_model*> ms(models, models + n_models);
  st = check_models(ctx, ms);
  if (st != RBMC_OK) return st;
  std::vector<const double*> zp(n_models, nullptr);
  std::vector<double*> dp(diag_out, diag_out + n_models), tp(n_models, nullptr);
  for (int j = 0; j < n_models; ++j) {
    if (!dp[j]) return fail(RBMC_E_ARG, "diag_out entry is NULL");
    if (opts->n_samples > 0) {
      if (!z || !z[j]) return fail(RBMC_E_UNSUPPORTED, "z must be supplied for every model");
      zp[j] = z[j];
    }
    if (opts->grad_mask) {
      if (!trace_out || !trace_out[j]) return fail(RBMC_E_ARG, "trace_out entry is NULL");
      tp[j] = trace_out[j];
    }
  }
  HIPCHK(hipSetDevice(ctx->device));
  double t0 = now_s();
  st = estimate_full(ctx, ms, opts, zp, dp, tp, rep);
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_ctx_get_tune(rbmc_ctx* ctx, rbmc_tune* t) {
  if (!ctx || !t) return fail(RBMC_E_ARG, "NULL argument");
  t->small_k = ctx->tune.small_k;
  t->small_tiles = ctx->tune.small_tiles;
  t->wide_from = ctx->tune.wide_from;
  return RBMC_OK;
}

rbmc_status rbmc_ctx_set_tune(rbmc_ctx* ctx, const rbmc_tune* t) {
  if (!ctx || !t) return fail(RBMC_E_ARG, "NULL argument");
  if (t->small_k < 0 || t->small_tiles < 0 || t->wide_from < kSweepWideFrom)
    return fail(RBMC_E_ARG, "small_k and small_tiles must be >= 0, wide_from >= 2048");
  ctx->tune.small_k = t->small_k;
  ctx->tune.small_tiles = t->small_tiles;
  ctx->tune.wide_from = t->wide_from;
  return RBMC_OK;
}


rbmc_status rbmc_autotune(rbmc_ctx* ctx, int32_t n_models, rbmc_model* const* models,
                          const rbmc_est_opts* opts, const double* const* z, const char* cache_path,
                          rbmc_tune_report* out) {
  if (!ctx || n_models < 1 || !models || !opts) return fail(RBMC_E_ARG, "NULL argument or no model");
  std::vector<rbmc_model*> ms(models, models + n_models);
  rbmc_status st = check_models(ctx, ms);
  if (st != RBMC_OK) return st;
  st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  HIPCHK(hipSetDevice(ctx->device));
  rbmc_tune_report rep{};
  const std::string sig = tune_signature(ctx, ms, opts), key = tune_key(sig);
  Tune cached;
  double cached_ms = 0.0;
  if (tune_cache_lookup(cache_path, key, &cached, &cached_ms)) {
    ctx->tune = cached;
    rep.best = rbmc_tune{cached.small_k, cached.small_tiles, cached.wide_from};
    rep.best_ms = cached_ms;
    rep.default_ms = -1.0;
    rep.from_cache = 1;
    if (out) *out = rep;
    return RBMC_OK;
  }
  // outputs of the timed runs (device diagonals, host traces)
  std::vector<double*> dp(n_models, nullptr), tp(n_models, nullptr);
  std::vector<std::vector<double>> th(n_models, std::vector<double>(4));
  Pool tmp;
  struct Release {
    Pool& p;
    ~Release() { p.release(); }
  } rel{tmp};
  for (int j = 0; j < n_models; ++j) {
    HIPCHK(tmp.alloc((void**)&dp[j], (size_t)ms[j]->plan.n * 8));
    tp[j] = th[j].data();
  }
  std::vector<Tune> cands;
  for (int wide : {kSweepWideFrom, INT_MAX})
    for (int sk : {256, 512})
      for (int stl : {768, 1536}) cands.push_back(Tune{sk, stl, wide});
  const Tune keep = ctx->tune;
  double best = 1e300;
  Tune best_t = cands[0];
  for (size_t i = 0; i < cands.size(); ++i) {
    ctx->tune = cands[i];
    double tmin = 1e300;
    for (int r = 0; r < 2; ++r) {  // a warm-up run, then a timed one
      for (rbmc_model* m : ms) m->bj_ready = m->sub_ready = false;
      HIPCHK(hipStreamSynchronize(ctx->stream));
      const double t0 = now_s();
      st = rbmc_estimate_batched(ctx, n_models, models, opts, z, dp.data(),
                                 opts->grad_mask ? tp.data() : nullptr, nullptr);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (st < 0) {
        ctx->tune = keep;
        return st;
      }
      if (r > 0) tmin = std::min(tmin, now_s() - t0);
    }
    if (i == 0) rep.default_ms = tmin * 1e3;
    if (tmin < best) {
      best = tmin;
      best_t = cands[i];
    }
  }
  ctx->tune = best_t;
  rep.best = rbmc_tune{best_t.small_k, best_t.small_tiles, best_t.wide_from};
  rep.best_ms = best * 1e3;
  rep.n_candidates = (int)cands.size();
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (f) {
      f << key << " " << best_t.small_k << " " << best_t.small_tiles << " " << best_t.wide_from
        << " " << rep.best_ms << " " << sig << "\n";
      rep.cache_written = f.good() ? 1 : 0;
    }
  }
  if (out) *out = rep;
  return RBMC_OK;
}

rbmc_status rbmc_precond_train(rbmc_model* m, const rbmc_est_opts* pcg_opts,
                               const rbmc_train_opts* train_opts, const double* z,
                               int32_t n_train, float* loss_out, rbmc_report* rep) {
  init_report(rep);
  if (!m || !pcg_opts || !train_opts || !z) return fail(RBMC_E_ARG, "NULL argument");
  if (n_train < 2) return fail(RBMC_E_ARG, "n_train must be >= 2 (a quarter of the columns is held out)");
  if (pcg_opts->pcg_maxit < 1 || !(pcg_opts->pcg_rtol > 0.0))
    return fail(RBMC_E_ARG, "pcg_maxit must be >= 1 and pcg_rtol > 0");
  if (train_opts->n_pairs < 2 || train_opts->epochs < 0 || train_opts->batch < 0)
    return fail(RBMC_E_ARG, "n_pairs must be >= 2, epochs and batch >= 0");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  rbmc_status st = precond_train(m, pcg_opts, train_opts, z, n_train, loss_out, rep);
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_precond_apply(rbmc_model* m, const double* r, const double* u, double* y,
                               int32_t n_rhs) {
  if (!m || !r || !u || !y) return fail(RBMC_E_ARG, "NULL argument");
  if (n_rhs < 0) return fail(RBMC_E_ARG, "n_rhs must be >= 0");
  if (!m->lrn.ready) return fail(RBMC_E_ARG, "the learned correction has no weights");
  if (n_rhs == 0) return RBMC_OK;
  HIPCHK(hipSetDevice(m->ctx->device));
  rbmc_status st = learned_apply(m->ctx, m, r, u, nullptr, nullptr, y, n_rhs, m->ctx->stream);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(m->ctx->stream));
  return RBMC_OK;
}

rbmc_status rbmc_precond_info(rbmc_model* m, rbmc_pc_info* info) {
  if (!m || !info) return fail(RBMC_E_ARG, "NULL argument");
  info->ready = m->lrn.ready ? 1 : 0;
  info->usable = learned_usable(m) ? 1 : 0;
  info->val_ratio = m->lrn.val_rel_err;
  info->trial_it_bj = m->lrn.trial_bj;
  info->trial_it_learned = m->lrn.trial_lrn;
  info->trial_s_bj = m->lrn.trial_s_bj;
  info->trial_s_learned = m->lrn.trial_s_lrn;
  return RBMC_OK;
}

rbmc_status rbmc_precond_get_weights(rbmc_model* m, float* w) {
  if (!m || !w) return fail(RBMC_E_ARG, "NULL argument");
  if (!m->lrn.ready) return fail(RBMC_E_ARG, "the learned correction has no weights");
  HIPCHK(hipSetDevice(m->ctx->device));
  HIPCHK(hipMemcpy(w, m->lrn.w, kNW * 4, hipMemcpyDeviceToHost));
  return RBMC_OK;
}

rbmc_status rbmc_precond_set_weights(rbmc_model* m, const float* w) {
  if (!m || !w) return fail(RBMC_E_ARG, "NULL argument");
  for (int i = 0; i < kNW; ++i)
    if (!std::isfinite(w[i])) return fail(RBMC_E_ARG, "weights must be finite");
  HIPCHK(hipSetDevice(m->ctx->device));
  rbmc_status st = ensure_learned(m);
  if (st != RBMC_OK) return st;
  HIPCHK(hipMemcpyAsync(m->lrn.w, w, kNW * 4, hipMemcpyHostToDevice, m->ctx->stream));
  learned_derive(m, m->ctx->stream);
  HIPCHK(hipStreamSynchronize(m->ctx->stream));
  m->lrn.ready = true;
  m->lrn.usable = true;  // weights given by the caller are taken as they are
  m->lrn.val_rel_err = -1.0;
  m->lrn.trial_bj = m->lrn.trial_lrn = -1;
  m->lrn.trial_s_bj = m->lrn.trial_s_lrn = -1.0;
  return RBMC_OK;
}

}  // extern "C"
