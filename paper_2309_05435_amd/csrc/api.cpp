// C ABI of the RBMC library and the host-side runtime that sequences the
// kernels: block-tridiagonal factorization of every chain (block-Jacobi cores
// and RBMC subdomains), the Takahashi sweep, the correction solves and the
// preconditioned conjugate-gradient sampler.
//
// Every launch works on all chains at once (grouped task lists), so a step
// of the recursion is one launch per kernel, not one per subdomain.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
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

struct ProfRec {
  int family;
  hipEvent_t a, b;
  double flops, bytes;
};

struct rbmc_ctx {
  int device;
  hipStream_t stream;
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;

  hipEvent_t ev() {
    hipEvent_t e = nullptr;
    if (!spare.empty()) {
      e = spare.back();
      spare.pop_back();
    } else {
      (void)hipEventCreate(&e);
    }
    return e;
  }
  // bracket a launch sequence of one kernel family
  int begin(int family, double flops, double bytes) {
    if (!prof) return -1;
    ProfRec r{family, ev(), ev(), flops, bytes};
    (void)hipEventRecord(r.a, stream);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id) {
    if (id >= 0) (void)hipEventRecord(recs[id].b, stream);
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
  }
};

namespace {

// Device allocations owned by a model.
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
      cap = std::max(host.size(), (size_t)1 << 20);
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

template <class T>
struct Launch {  // a grouped launch: task offset, count, tiles
  size_t off = 0;
  int n = 0;
  int tiles = 0;
};

struct ChainSet {
  std::vector<Chain> chains;
  std::vector<int> np;             // padded block size per chain
  std::vector<double*> S;          // T x np^2, S_t^-1 after factorization
  std::vector<double*> tmp;        // np^2 (Schur / Takahashi temporaries)
  std::vector<double*> sig, xb;    // np^2 (Takahashi Sigma and X), subdomains only
  std::vector<double*> gjU, gjB;   // np x 256 Gauss-Jordan panels
  std::vector<double*> gjP, gjPi;  // 256 x 256 outer pivot block, 64 x 64 inner pivot inverse
  std::vector<double*> gjUi, gjBi; // 256 x 64 inner panels
  int maxT = 0;
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
  Pool work;      // sample-count dependent workspace
  int work_nk = -1;
  DevModel dm{};
  double *d_qs = nullptr, *d_kk = nullptr, *d_fs = nullptr, *d_qd = nullptr, *d_dqd = nullptr,
         *d_ld = nullptr, *d_dvec = nullptr;
  int* d_obs_rank = nullptr;
  std::vector<RegionDev> regions;
  RegionDev* d_regions = nullptr;
  uint8_t** d_inbox = nullptr;
  ChainSet bj, sub;
  int* d_info = nullptr;  // one per chain: bj then sub
  bool bj_ready = false, sub_ready = false;
  // workspace (n_k dependent)
  double *w_r = nullptr, *w_p = nullptr, *w_q = nullptr, *w_z = nullptr, *w_x = nullptr;
  double* w_scal = nullptr;  // 8 x n_k per-column scalars
  double* w_part = nullptr;  // partial sums
  uint8_t* w_active = nullptr;
  int* w_iters = nullptr;    // n_k + 1
  std::vector<std::vector<double*>> bj_pan, sub_pan;  // per chain: T panels np x n_k
  std::vector<double*> bj_y, sub_y;                  // per chain temp panel
  double* w_diag_part = nullptr;
  size_t diag_part_len = 0;
  Arena arena;
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
  HIPCHK(hipStreamSynchronize(s));
  m->dm.qo = c.qo;
  m->dm.dqo = c.dqo;
  m->dm.lo = c.lo;
  m->bj_ready = m->sub_ready = false;
  return RBMC_OK;
}

bool theta_ok(double lk, double lt, double rho, double ls) {
  return std::isfinite(lk) && std::isfinite(lt) && std::isfinite(rho) && std::isfinite(ls) &&
         std::fabs(rho) < 1.0;
}

rbmc_status alloc_chainset(rbmc_model* m, ChainSet& cs, const std::vector<Chain>& chains,
                           bool subdomains) {
  cs.chains = chains;
  cs.maxT = 0;
  for (const Chain& c : chains) {
    const int np = pad_to(m->plan.regions[c.region].nb());
    cs.np.push_back(np);
    const size_t blk = (size_t)np * np;
    double* p = nullptr;
    HIPCHK(m->pool.alloc((void**)&p, blk * c.T * 8));
    cs.S.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, blk * 8));
    cs.tmp.push_back(p);
    if (subdomains) {
      HIPCHK(m->pool.alloc((void**)&p, blk * 8));
      cs.sig.push_back(p);
      HIPCHK(m->pool.alloc((void**)&p, blk * 8));
      cs.xb.push_back(p);
    }
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * 256 * 8));
    cs.gjU.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)np * 256 * 8));
    cs.gjB.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)256 * 256 * 8));
    cs.gjP.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)64 * 64 * 8));
    cs.gjPi.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)256 * 64 * 8));
    cs.gjUi.push_back(p);
    HIPCHK(m->pool.alloc((void**)&p, (size_t)256 * 64 * 8));
    cs.gjBi.push_back(p);
    cs.maxT = std::max(cs.maxT, c.T);
  }
  return RBMC_OK;
}

rbmc_status ensure_work(rbmc_model* m, int n_k) {
  if (m->work_nk >= n_k && m->work_nk >= 1) return RBMC_OK;
  m->work.release();
  m->work_nk = -1;
  m->w_diag_part = nullptr;
  m->diag_part_len = 0;
  const int nk = std::max(n_k, 1);
  const size_t vec = (size_t)m->plan.n * nk * 8;
  HIPCHK(m->work.alloc((void**)&m->w_r, vec));
  HIPCHK(m->work.alloc((void**)&m->w_p, vec));
  HIPCHK(m->work.alloc((void**)&m->w_q, vec));
  HIPCHK(m->work.alloc((void**)&m->w_z, vec));
  HIPCHK(m->work.alloc((void**)&m->w_x, vec));
  HIPCHK(m->work.alloc((void**)&m->w_scal, (size_t)8 * nk * 8));
  const int nch = std::max(spmm_chunks(m->dm), dot_chunks(m->plan.n));
  HIPCHK(m->work.alloc((void**)&m->w_part, (size_t)nch * nk * 8));
  HIPCHK(m->work.alloc((void**)&m->w_active, (size_t)nk));
  HIPCHK(m->work.alloc((void**)&m->w_iters, (size_t)(nk + 1) * 4));
  auto panels = [&](ChainSet& cs, std::vector<std::vector<double*>>& pan,
                    std::vector<double*>& ytmp) -> rbmc_status {
    pan.assign(cs.chains.size(), {});
    ytmp.assign(cs.chains.size(), nullptr);
    for (size_t c = 0; c < cs.chains.size(); ++c) {
      const size_t psz = (size_t)cs.np[c] * nk * 8;
      for (int t = 0; t < cs.chains[c].T; ++t) {
        double* p = nullptr;
        HIPCHK(m->work.alloc((void**)&p, psz));
        pan[c].push_back(p);
      }
      HIPCHK(m->work.alloc((void**)&ytmp[c], psz));
    }
    return RBMC_OK;
  };
  rbmc_status st = panels(m->bj, m->bj_pan, m->bj_y);
  if (st != RBMC_OK) return st;
  st = panels(m->sub, m->sub_pan, m->sub_y);
  if (st != RBMC_OK) return st;
  m->work_nk = nk;
  return RBMC_OK;
}

// ---- task builders ----------------------------------------------------------

int gemm_tiles(int M, int N) { return ((M + 127) / 128) * ((N + 127) / 128); }

struct GemmList {
  std::vector<GemmTask> v;
  int tiles = 0;
  double flops = 0.0;  // algorithmic (unpadded) flops of the list
  void add(const double* A, const double* B, const double* Cin, double* C, int M, int N, int K,
           int lda, int ldb, int ldc, double alpha, double beta, int tA, int tB, int Mreal,
           int Kreal) {
    flops += 2.0 * Mreal * (double)N * Kreal;
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
    t.tiles_n = (N + 127) / 128;
    t.tile_start = tiles;
    tiles += gemm_tiles(M, N);
    v.push_back(t);
  }
  // restrict the last product to the lower 128-tiles of a square result
  void set_last_lower() {
    GemmTask& t = v.back();
    tiles -= gemm_tiles(t.M, t.N);
    tiles += gemm_task_tiles(t.M, t.N, 1);
    t.lower = 1;
  }
  // outer sweep update of the lower tiles: M -= U B^T outside rows/cols [kb, kb + w)
  void add_sweep(double* Mx, int np, const double* U, const double* B, int w, int kb) {
    GemmTask t{};
    t.A = U;
    t.B = B;
    t.Cin = Mx;
    t.C = Mx;
    t.M = np;
    t.N = np;
    t.K = w;
    t.lda = np;
    t.ldb = np;
    t.ldc = np;
    t.ldcin = np;
    t.alpha = -1.0;
    t.beta = 1.0;
    t.transA = 0;
    t.transB = 1;
    t.tiles_n = (np + 127) / 128;
    t.lower = 1;
    t.skip0 = kb;
    t.skip1 = kb + w;
    t.tile_start = tiles;
    tiles += gemm_task_tiles(np, np, 1);
    v.push_back(t);
  }
};

struct StencilList {
  std::vector<StencilTask> v;
  int tiles = 0;
  double bytes = 0.0;
  int max_sparse_np = 0;  // largest block with sparse terms (0: none)
  void add(StencilTask t, int np, int nb) {
    t.tile_start = tiles;
    tiles += (np / 64) * ((t.ncols + 63) / 64);
    bytes += 16.0 * nb * (double)t.ncols;
    if (t.gamma != 0.0 || t.dv != nullptr || t.pad_identity) max_sparse_np = std::max(max_sparse_np, np);
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

// Recorded program: a sequence of grouped launches over the arena.
struct InvJob {  // one SPD block to invert in place, with its workspace
  double* M;
  int np, nb;
  int* info;
  double *B, *U, *P, *Pi, *Ui, *Bi;
};

struct Op {
  // 0 gemm, 1 stencil, 2 sweep step (rank 64), 3 panels, 4 extract, 5 mc, 6 copy,
  // 7 outer gather, 8 outer fix, 9 sweep finish, 10 profile begin, 11 profile end
  int kind;
  size_t off;
  int n, tiles;
  int max_np = 0, kblk = 0;
  const double* X = nullptr;
  double* Xout = nullptr;
  int n_k = 0;
  // copy
  void* dst = nullptr;
  const void* src = nullptr;
  size_t bytes = 0;
  // instrumentation: kernel family and algorithmic work of the launch
  int family = -1;
  double alg_flops = 0.0, alg_bytes = 0.0;
};

struct Program {
  std::vector<Op> ops;
  void gemm(Arena& a, GemmList& g, bool profiled = true) {
    if (g.v.empty()) return;
    Op o;
    o.kind = 0;
    o.off = a.push(g.v);
    o.n = (int)g.v.size();
    o.tiles = g.tiles;
    o.family = profiled ? RBMC_KF_GEMM : -1;
    o.alg_flops = g.flops;
    ops.push_back(std::move(o));
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
    ops.push_back(std::move(o));
  }
  void mirror(Arena& a, const std::vector<InvTask>& t) {
    if (t.empty()) return;
    Op o;
    o.kind = 12;
    o.off = a.push(t);
    o.n = (int)t.size();
    for (const InvTask& it : t) o.max_np = std::max(o.max_np, it.np);
    ops.push_back(std::move(o));
  }
  // rank-64 sweep of a list of blocks (all steps) followed by the finish pass
  void sweep64(Arena& a, const std::vector<InvTask>& t) {
    if (t.empty()) return;
    const size_t off = a.push(t);
    int max_np = 0;
    for (const InvTask& it : t) max_np = std::max(max_np, it.np);
    for (int k = 0; k < max_np / 64; ++k) {
      Op o;
      o.kind = 2;
      o.off = off;
      o.n = (int)t.size();
      o.max_np = max_np;
      o.kblk = k;
      ops.push_back(std::move(o));
    }
    Op f;
    f.kind = 9;
    f.off = off;
    f.n = (int)t.size();
    ops.push_back(std::move(f));
  }
  // In-place inversion of SPD blocks: blocks up to 256 by the rank-64 sweep;
  // larger ones by rank-256 outer sweeps (GEMM updates) whose 256 x 256 pivot
  // blocks are inverted by the rank-64 sweep.
  void inverse(Arena& a, const std::vector<InvJob>& jobs) {
    if (jobs.empty()) return;
    Op pb;
    pb.kind = 10;
    pb.family = RBMC_KF_SPD_INVERSE;
    for (const InvJob& j : jobs) pb.alg_flops += (double)j.nb * j.nb * j.nb;
    ops.push_back(pb);
    std::vector<InvTask> small, big;
    int max_big = 0;
    for (const InvJob& j : jobs) {
      InvTask t{};
      t.M = j.M;
      t.np = j.np;
      t.nb = j.nb;
      t.info = j.info;
      t.U = j.U;
      t.Bp = j.B;
      t.Pi = j.Pi;
      if (j.np <= 256) small.push_back(t);
      else {
        big.push_back(t);
        max_big = std::max(max_big, j.np);
      }
    }
    sweep64(a, small);
    for (int kb = 0; kb < max_big; kb += 256) {
      TileList<Gj2Task> gl;
      std::vector<InvTask> inner;
      GemmList gu, gm;
      for (const InvJob& j : jobs) {
        if (j.np <= 256 || kb >= j.np) continue;
        const int w = std::min(256, j.np - kb);
        Gj2Task g{};
        g.M = j.M;
        g.B = j.B;
        g.U = j.U;
        g.P = j.P;
        g.np = j.np;
        g.kb = kb;
        g.w = w;
        gl.add(g, gj2_tiles(j.np, w));
        InvTask t{};
        t.M = j.P;
        t.np = w;
        t.nb = w;
        t.info = j.info;
        t.U = j.Ui;
        t.Bp = j.Bi;
        t.Pi = j.Pi;
        inner.push_back(t);
        // U = B P^-1
        gu.add(j.B, j.P, nullptr, j.U, j.np, w, w, j.np, w, j.np, 1.0, 0.0, 0, 0, j.np, w);
        // M_lower -= U B^T outside the swept block row/column
        gm.add_sweep(j.M, j.np, j.U, j.B, w, kb);
      }
      Op og;
      og.kind = 7;
      og.off = a.push(gl.v);
      og.n = (int)gl.v.size();
      og.tiles = gl.tiles;
      ops.push_back(std::move(og));
      sweep64(a, inner);
      gemm(a, gu, false);
      gemm(a, gm, false);
      Op of;
      of.kind = 8;
      of.off = og.off;
      of.n = og.n;
      of.tiles = og.tiles;
      ops.push_back(std::move(of));
    }
    if (!big.empty()) {
      Op f;
      f.kind = 9;
      f.off = a.push(big);
      f.n = (int)big.size();
      ops.push_back(std::move(f));
    }
    Op pe;
    pe.kind = 11;
    ops.push_back(pe);
  }
  void panels(Arena& a, TileList<PanelTask>& p, const double* X, double* Xout, int n_k) {
    if (p.v.empty()) return;
    Op o;
    o.kind = 3;
    o.off = a.push(p.v);
    o.n = (int)p.v.size();
    o.tiles = p.tiles;
    o.family = RBMC_KF_PANELS;
    o.alg_bytes = p.bytes;
    o.X = X;
    o.Xout = Xout;
    o.n_k = n_k;
    ops.push_back(std::move(o));
  }
  void extract(Arena& a, TileList<ExtractTask>& e) {
    if (e.v.empty()) return;
    Op o;
    o.kind = 4;
    o.off = a.push(e.v);
    o.n = (int)e.v.size();
    o.tiles = e.tiles;
    ops.push_back(std::move(o));
  }
  void mc(Arena& a, TileList<McTask>& e, int n_k) {
    if (e.v.empty()) return;
    Op o;
    o.kind = 5;
    o.off = a.push(e.v);
    o.n = (int)e.v.size();
    o.tiles = e.tiles;
    o.n_k = n_k;
    ops.push_back(std::move(o));
  }
  void copy(void* dst, const void* src, size_t bytes) {
    Op o;
    o.kind = 6;
    o.dst = dst;
    o.src = src;
    o.bytes = bytes;
    ops.push_back(std::move(o));
  }
};

struct RunCtx {
  double* diag_out = nullptr;
  double* partial = nullptr;
  int nchunk_max = 0;
};

rbmc_status run(rbmc_model* m, const Program& pg, const RunCtx& rc) {
  hipStream_t s = m->ctx->stream;
  Arena& a = m->arena;
  std::vector<int> open_prof;  // records opened by profile-begin ops
  for (const Op& o : pg.ops) {
    const int pid = (o.family >= 0) ? m->ctx->begin(o.family, o.alg_flops, o.alg_bytes) : -1;
    switch (o.kind) {
      case 0: launch_gemm(a.at<GemmTask>(o.off), o.n, o.tiles, s); break;
      case 1:
        launch_rstencil(a.at<StencilTask>(o.off), o.n, o.tiles, m->d_regions, m->d_qs,
                        m->plan.ns, o.max_np, s);
        break;
      case 12: launch_mirror(a.at<InvTask>(o.off), o.n, o.max_np, s); break;
      case 2: launch_gj_step(a.at<InvTask>(o.off), o.n, o.max_np, o.kblk, s); break;
      case 7: launch_gj2_gather(a.at<Gj2Task>(o.off), o.n, o.tiles, s); break;
      case 8: launch_gj2_fix(a.at<Gj2Task>(o.off), o.n, o.tiles, s); break;
      case 9: launch_gj_finish(a.at<InvTask>(o.off), o.n, s); break;
      case 10: open_prof.push_back(pid); break;
      case 11:
        if (!open_prof.empty()) {
          m->ctx->end(open_prof.back());
          open_prof.pop_back();
        }
        break;
      case 3:
        launch_panels(a.at<PanelTask>(o.off), o.n, o.tiles, m->d_regions, m->dm, o.X, o.Xout,
                      o.n_k, s);
        break;
      case 4:
        launch_extract(a.at<ExtractTask>(o.off), o.n, o.tiles, m->d_regions, m->d_inbox, m->dm,
                       rc.diag_out, rc.partial, rc.nchunk_max, s);
        break;
      case 5:
        launch_mc(a.at<McTask>(o.off), o.n, o.tiles, m->d_regions, m->d_inbox, m->dm, o.n_k,
                  rc.diag_out, rc.partial, rc.nchunk_max, s);
        break;
      case 6: HIPCHK(hipMemcpyAsync(o.dst, o.src, o.bytes, hipMemcpyDeviceToDevice, s)); break;
    }
    if (o.kind != 10) m->ctx->end(pid);
  }
  HIPCHK(hipGetLastError());
  return RBMC_OK;
}

// Factorization program: S_t^-1 of every chain of the set.
//   S_0 = B_0,  S_t = B_t - q_o^2 Q_R S_{t-1}^-1 Q_R,  B_t = q_d(t) Q_R + D_t
void build_factor(rbmc_model* m, ChainSet& cs, int info_base, Program& pg) {
  Arena& a = m->arena;
  for (int t = 0; t < cs.maxT; ++t) {
    StencilList v1, v2;
    std::vector<InvJob> inv;
    for (size_t c = 0; c < cs.chains.size(); ++c) {
      const Chain& ch = cs.chains[c];
      if (t >= ch.T) continue;
      const int np = cs.np[c];
      const size_t blk = (size_t)np * np;
      const int tg = ch.t0 + t;
      double* St = cs.S[c] + blk * t;
      if (t > 0) {
        StencilTask s1{};
        s1.M = cs.S[c] + blk * (t - 1);
        s1.ldm = np;
        s1.out = cs.tmp[c];
        s1.ldout = np;
        s1.ncols = np;
        s1.alpha = 1.0;
        s1.region = ch.region;
        v1.add(s1, np, m->regions[ch.region].nb);
      }
      StencilTask s2{};
      s2.M = (t > 0) ? cs.tmp[c] : nullptr;
      s2.ldm = np;
      s2.trans = 1;
      s2.alpha = (t > 0) ? -m->co.qo * m->co.qo : 0.0;
      s2.gamma = m->co.qd[tg];
      s2.dv = m->d_dvec + (size_t)tg * m->plan.ns;
      s2.pad_identity = 1;
      s2.out = St;
      s2.ldout = np;
      s2.ncols = np;
      s2.region = ch.region;
      v2.add(s2, np, m->regions[ch.region].nb);
      InvJob it{};
      it.M = St;
      it.np = np;
      it.nb = m->regions[ch.region].nb;
      it.info = m->d_info + info_base + (int)c;
      it.B = cs.gjB[c];
      it.U = cs.gjU[c];
      it.P = cs.gjP[c];
      it.Pi = cs.gjPi[c];
      it.Ui = cs.gjUi[c];
      it.Bi = cs.gjBi[c];
      inv.push_back(it);
    }
    pg.stencil(a, v1);
    pg.stencil(a, v2);
    pg.inverse(a, inv);
  }
}

// Block-tridiagonal solve with the chain factors, in place on the panels:
// forward u_0 = S_0^-1 r_0, u_t = S_t^-1 (r_t - q_o Q_R u_{t-1});
// backward z_t = u_t - S_t^-1 (q_o Q_R z_{t+1}) down to local step stop[c].
// r_0 must be in ytmp[c], r_t (t >= 1) in pan[c][t].
void build_solve(rbmc_model* m, ChainSet& cs, std::vector<std::vector<double*>>& pan,
                 std::vector<double*>& ytmp, int n_k, const std::vector<int>& stop,
                 Program& pg) {
  Arena& a = m->arena;
  const double qo = m->co.qo;
  for (int t = 0; t < cs.maxT; ++t) {
    StencilList sl;
    GemmList gl;
    for (size_t c = 0; c < cs.chains.size(); ++c) {
      const Chain& ch = cs.chains[c];
      if (t >= ch.T) continue;
      const int np = cs.np[c];
      const size_t blk = (size_t)np * np;
      if (t > 0) {
        StencilTask s{};
        s.M = pan[c][t - 1];
        s.ldm = np;
        s.In = pan[c][t];
        s.ldin = np;
        s.beta = 1.0;
        s.alpha = -qo;
        s.out = ytmp[c];
        s.ldout = np;
        s.ncols = n_k;
        s.region = ch.region;
        sl.add(s, np, m->regions[ch.region].nb);
      }
      gl.add(cs.S[c] + blk * t, ytmp[c], nullptr, pan[c][t], np, n_k, np, np, np, np, 1.0, 0.0, 1, 0, m->regions[ch.region].nb, m->regions[ch.region].nb);
    }
    pg.stencil(a, sl);
    pg.gemm(a, gl);
  }
  for (int t = cs.maxT - 2; t >= 0; --t) {
    StencilList sl;
    GemmList gl;
    for (size_t c = 0; c < cs.chains.size(); ++c) {
      const Chain& ch = cs.chains[c];
      if (t > ch.T - 2 || t < stop[c]) continue;
      const int np = cs.np[c];
      const size_t blk = (size_t)np * np;
      StencilTask s{};
      s.M = pan[c][t + 1];
      s.ldm = np;
      s.alpha = qo;
      s.out = ytmp[c];
      s.ldout = np;
      s.ncols = n_k;
      s.region = ch.region;
      sl.add(s, np, m->regions[ch.region].nb);
      gl.add(cs.S[c] + blk * t, ytmp[c], pan[c][t], pan[c][t], np, n_k, np, np, np, np, -1.0,
             1.0, 1, 0, m->regions[ch.region].nb, m->regions[ch.region].nb);
    }
    pg.stencil(a, sl);
    pg.gemm(a, gl);
  }
}

rbmc_status check_info(rbmc_model* m, int base, int count, rbmc_report* rep, const char* what) {
  std::vector<int> info(count);
  if (count == 0) return RBMC_OK;
  HIPCHK(hipMemcpy(info.data(), m->d_info + base, count * 4, hipMemcpyDeviceToHost));
  for (int c = 0; c < count; ++c)
    if (info[c] != 0) {
      if (rep) {
        rep->fail_subdomain = c;
        rep->fail_block = info[c] - 1;
      }
      return fail(RBMC_E_NOT_SPD, std::string(what) + " chain " + std::to_string(c) +
                                      " lost positive definiteness");
    }
  return RBMC_OK;
}

rbmc_status factor_set(rbmc_model* m, ChainSet& cs, int info_base, rbmc_report* rep,
                       const char* what) {
  hipStream_t s = m->ctx->stream;
  HIPCHK(hipMemsetAsync(m->d_info + info_base, 0, cs.chains.size() * 4, s));
  m->arena.clear();
  Program pg;
  build_factor(m, cs, info_base, pg);
  HIPCHK(m->arena.upload(s));
  rbmc_status st = run(m, pg, RunCtx{});
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  return check_info(m, info_base, (int)cs.chains.size(), rep, what);
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
  if (o->precision != RBMC_FP64) return fail(RBMC_E_UNSUPPORTED, "only RBMC_FP64 is built");
  if (o->precond != RBMC_PC_BJ) return fail(RBMC_E_UNSUPPORTED, "only RBMC_PC_BJ is built");
  return RBMC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
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
  rbmc_ctx* c = new rbmc_ctx;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return RBMC_OK;
}

void rbmc_ctx_destroy(rbmc_ctx* ctx) { delete ctx; }

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
    m->work.release();
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
  {
    std::vector<int> rank(P.n, -1);
    int r = 0;
    for (int i = 0; i < P.n; ++i)
      if (m->mask[i]) rank[i] = r++;
    MCHK(hipMemcpy(m->d_obs_rank, rank.data(), (size_t)P.n * 4, hipMemcpyHostToDevice));
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
  // regions
  std::vector<uint8_t*> inbox_ptrs;
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
    m->regions.push_back(rd);
    inbox_ptrs.push_back(ib);
  }
  MCHK(m->pool.alloc((void**)&m->d_regions, m->regions.size() * sizeof(RegionDev)));
  MCHK(hipMemcpy(m->d_regions, m->regions.data(), m->regions.size() * sizeof(RegionDev),
                 hipMemcpyHostToDevice));
  MCHK(m->pool.alloc((void**)&m->d_inbox, inbox_ptrs.size() * sizeof(uint8_t*)));
  MCHK(hipMemcpy(m->d_inbox, inbox_ptrs.data(), inbox_ptrs.size() * sizeof(uint8_t*),
                 hipMemcpyHostToDevice));
  MCHK(m->pool.alloc((void**)&m->d_info, (P.bj.size() + P.sub.size()) * 4));
  {
    rbmc_status st = alloc_chainset(m, m->bj, P.bj, false);
    if (st != RBMC_OK) return cleanup(st);
    st = alloc_chainset(m, m->sub, P.sub, true);
    if (st != RBMC_OK) return cleanup(st);
    st = upload_coefs(m);
    if (st != RBMC_OK) return cleanup(st);
  }
#undef MCHK
  *out = m;
  return RBMC_OK;
}

void rbmc_model_destroy(rbmc_model* m) {
  if (!m) return;
  (void)hipSetDevice(m->ctx->device);
  m->work.release();
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
  HIPCHK(hipSetDevice(m->ctx->device));
  launch_apply_op(m->dm, op, x, y, n_rhs, m->ctx->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(m->ctx->stream));
  return RBMC_OK;
}

// Block-Jacobi PCG on Q x = F z for all samples at once.
static rbmc_status sample_impl(rbmc_model* m, const rbmc_est_opts* o, const double* z, double* x,
                               rbmc_report* rep) {
  const int n = m->plan.n, nk = o->n_samples;
  hipStream_t s = m->ctx->stream;
  double t0 = now_s();
  if (!m->bj_ready) {
    rbmc_status st = factor_set(m, m->bj, 0, rep, "block-Jacobi");
    if (st != RBMC_OK) return st;
    m->bj_ready = true;
  }
  rbmc_status st = ensure_work(m, nk);
  if (st != RBMC_OK) return st;
  double* r = m->w_r;
  double* p = m->w_p;
  double* q = m->w_q;
  double* zz = m->w_z;
  double* bb = m->w_scal;
  double* rz = m->w_scal + nk;
  double* rzn = m->w_scal + 2 * nk;
  double* pq = m->w_scal + 3 * nk;
  double* rr = m->w_scal + 4 * nk;
  const int nch = dot_chunks(n), nsp = spmm_chunks(m->dm);
  // preconditioner program: gather r -> panels, solve, scatter -> z
  m->arena.clear();
  Program pre, gat, sca;
  TileList<PanelTask> g, sc;
  for (size_t c = 0; c < m->bj.chains.size(); ++c) {
    const Chain& ch = m->bj.chains[c];
    const int np = m->bj.np[c];
    for (int t = 0; t < ch.T; ++t) {
      PanelTask pt{};
      pt.P = (t == 0) ? m->bj_y[c] : m->bj_pan[c][t];
      pt.region = ch.region;
      pt.t = ch.t0 + t;
      pt.mode = 0;
      g.add(pt, panel_tiles(np, nk), 16.0 * m->regions[ch.region].nb * nk);
      PanelTask ps = pt;
      ps.P = m->bj_pan[c][t];
      ps.mode = 1;
      sc.add(ps, panel_tiles(np, nk), 16.0 * m->regions[ch.region].nb * nk);
    }
  }
  gat.panels(m->arena, g, r, nullptr, nk);
  std::vector<int> stop(m->bj.chains.size(), 0);
  build_solve(m, m->bj, m->bj_pan, m->bj_y, nk, stop, pre);
  sca.panels(m->arena, sc, nullptr, zz, nk);
  HIPCHK(m->arena.upload(s));
  auto precond = [&]() -> rbmc_status {
    rbmc_status e = run(m, gat, RunCtx{});
    if (e != RBMC_OK) return e;
    e = run(m, pre, RunCtx{});
    if (e != RBMC_OK) return e;
    return run(m, sca, RunCtx{});
  };
  // b = F z -> r; x = 0
  launch_apply_op(m->dm, RBMC_OP_F, z, r, nk, s);
  HIPCHK(hipMemsetAsync(x, 0, (size_t)n * nk * 8, s));
  launch_dot_partials(r, r, n, nk, m->w_part, nch, s);
  launch_reduce_partials(m->w_part, nch, nk, bb, s);
  std::vector<double> hbb(nk);
  HIPCHK(hipMemcpyAsync(hbb.data(), bb, (size_t)nk * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint8_t> act(nk);
  for (int k = 0; k < nk; ++k) act[k] = hbb[k] > 0.0;
  HIPCHK(hipMemcpyAsync(m->w_active, act.data(), nk, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(m->w_iters, 0, (size_t)(nk + 1) * 4, s));
  st = precond();
  if (st != RBMC_OK) return st;
  launch_dot_partials(r, zz, n, nk, m->w_part, nch, s);
  launch_reduce_partials(m->w_part, nch, nk, rz, s);
  launch_pcg_p(zz, p, rz, rz, m->w_active, n, nk, 1, s);
  int n_active = 0;
  for (int k = 0; k < nk; ++k) n_active += act[k];
  int it = 0;
  while (n_active > 0 && it < o->pcg_maxit) {
    const int pid = m->ctx->begin(RBMC_KF_SPMM, 0.0, 16.0 * n * (double)nk);
    launch_spmm_dot(m->dm, p, q, m->w_part, nk, s);
    m->ctx->end(pid);
    launch_reduce_partials(m->w_part, nsp, nk, pq, s);
    launch_pcg_xr(p, q, x, r, rz, pq, m->w_active, n, nk, m->w_part, nch, s);
    launch_reduce_partials(m->w_part, nch, nk, rr, s);
    launch_pcg_check(rr, bb, o->pcg_rtol, m->w_active, m->w_iters + 1, m->w_iters, nk, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&n_active, m->w_iters, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ++it;
    if (n_active == 0) break;
    st = precond();
    if (st != RBMC_OK) return st;
    launch_dot_partials(r, zz, n, nk, m->w_part, nch, s);
    launch_reduce_partials(m->w_part, nch, nk, rzn, s);
    launch_pcg_p(zz, p, rzn, rz, m->w_active, n, nk, 0, s);
  }
  HIPCHK(hipGetLastError());
  std::vector<int> iters(nk + 1);
  std::vector<double> hrr(nk);
  HIPCHK(hipMemcpyAsync(iters.data(), m->w_iters, (size_t)(nk + 1) * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hrr.data(), rr, (size_t)nk * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (rep) {
    int itmax = 0;
    double itsum = 0.0, maxres = 0.0;
    for (int k = 0; k < nk; ++k) {
      itmax = std::max(itmax, iters[k + 1]);
      itsum += iters[k + 1];
      if (hbb[k] > 0.0) maxres = std::max(maxres, std::sqrt(hrr[k] / hbb[k]));
    }
    rep->pcg_it_max = itmax;
    rep->pcg_it_mean = nk ? itsum / nk : 0.0;
    rep->max_rel_residual = maxres;
    rep->t_sample = now_s() - t0;
    rep->peak_bytes = m->pool.bytes + m->work.bytes;
  }
  return n_active > 0 ? RBMC_W_NOT_CONVERGED : RBMC_OK;
}

// Estimator from samples x (n x n_k, device).
static rbmc_status estimate_impl(rbmc_model* m, const rbmc_est_opts* o, const double* x,
                                 double* diag_out, double* trace_out, rbmc_report* rep) {
  const int nk = o->n_samples;
  hipStream_t s = m->ctx->stream;
  const Plan& P = m->plan;
  double t0 = now_s();
  if (!m->sub_ready) {
    rbmc_status st = factor_set(m, m->sub, (int)m->bj.chains.size(), rep, "subdomain");
    if (st != RBMC_OK) return st;
    m->sub_ready = true;
  }
  double t1 = now_s();
  rbmc_status st = ensure_work(m, nk);
  if (st != RBMC_OK) return st;
  ChainSet& cs = m->sub;
  const int nchains = (int)cs.chains.size();
  // trace slots: per chain, per local step: det (diag block, off t->t+1, off t+1->t) and mc
  int nchunk_max = 1;
  for (int c = 0; c < nchains; ++c) nchunk_max = std::max(nchunk_max, (cs.np[c] + 255) / 256);
  std::vector<int> slot_base(nchains + 1, 0);
  for (int c = 0; c < nchains; ++c) slot_base[c + 1] = slot_base[c] + cs.chains[c].T * 4;
  const int nslots = slot_base[nchains];
  const int mc_chunks = [&] {
    int v = 1;
    for (int c = 0; c < nchains; ++c) v = std::max(v, cs.np[c] / 64);
    return v;
  }();
  const size_t det_len = (size_t)nslots * nchunk_max * 3;
  const size_t mc_len = (size_t)nslots * mc_chunks * 8;
  const size_t need = det_len + mc_len;
  if (m->diag_part_len < need) {
    double* p = nullptr;
    HIPCHK(m->work.alloc((void**)&p, need * 8));
    m->w_diag_part = p;
    m->diag_part_len = need;
  }
  double* det_part = m->w_diag_part;
  double* mc_part = m->w_diag_part + det_len;
  HIPCHK(hipMemsetAsync(m->w_diag_part, 0, need * 8, s));

  // ---- Takahashi sweep ----
  m->arena.clear();
  Program tak;
  auto lc0 = [&](int c) { return cs.chains[c].ct0 - cs.chains[c].t0; };
  auto lc1 = [&](int c) { return lc0(c) + cs.chains[c].cT - 1; };
  auto is_core = [&](int c, int t) { return t >= lc0(c) && t <= lc1(c); };
  {
    TileList<ExtractTask> ex;
    for (int c = 0; c < nchains; ++c) {
      const Chain& ch = cs.chains[c];
      const int np = cs.np[c];
      const size_t blk = (size_t)np * np;
      tak.copy(cs.sig[c], cs.S[c] + blk * (ch.T - 1), blk * 8);
      if (is_core(c, ch.T - 1)) {
        ExtractTask e{};
        e.M = cs.sig[c];
        e.ld = np;
        e.region = ch.region;
        e.t = ch.t0 + ch.T - 1;
        e.kind = 0;
        e.sign = 1.0;
        e.out_slot = slot_base[c] + (ch.T - 1) * 4 + 0;
        ex.add(e, (np + 255) / 256);
      }
    }
    tak.extract(m->arena, ex);
  }
  for (int t = cs.maxT - 2; t >= 0; --t) {
    StencilList s1, s2;
    GemmList g1, g2;
    TileList<ExtractTask> e1, e2;
    std::vector<InvTask> mir;
    for (int c = 0; c < nchains; ++c) {
      const Chain& ch = cs.chains[c];
      if (t > ch.T - 2) continue;
      const int stop_x = std::max(lc0(c) - 1, 0);
      if (t < stop_x) continue;
      const int np = cs.np[c];
      const size_t blk = (size_t)np * np;
      StencilTask v{};
      v.M = cs.sig[c];
      v.ldm = np;
      v.alpha = 1.0;
      v.out = cs.tmp[c];
      v.ldout = np;
      v.ncols = np;
      v.region = ch.region;
      s1.add(v, np, m->regions[ch.region].nb);
      // X = q_o V^T S_t^-1  (Sigma_{t+1,t} = -X)
      g1.add(cs.tmp[c], cs.S[c] + blk * t, nullptr, cs.xb[c], np, np, np, np, np, np, m->co.qo,
             0.0, 1, 0, m->regions[ch.region].nb, m->regions[ch.region].nb);
      if (is_core(c, t)) {  // rows at t, columns at t+1: Sigma_{t,t+1} = -X^T
        ExtractTask e{};
        e.M = cs.xb[c];
        e.ld = np;
        e.region = ch.region;
        e.t = ch.t0 + t;
        e.kind = 1;
        e.trans = 1;
        e.sign = -1.0;
        e.out_slot = slot_base[c] + t * 4 + 1;
        e1.add(e, (np + 255) / 256);
      }
      if (is_core(c, t + 1)) {  // rows at t+1, columns at t: Sigma_{t+1,t} = -X
        ExtractTask e{};
        e.M = cs.xb[c];
        e.ld = np;
        e.region = ch.region;
        e.t = ch.t0 + t + 1;
        e.kind = 1;
        e.trans = 0;
        e.sign = -1.0;
        e.out_slot = slot_base[c] + (t + 1) * 4 + 2;
        e1.add(e, (np + 255) / 256);
      }
      if (t >= lc0(c)) {
        StencilTask z{};
        z.M = cs.xb[c];
        z.ldm = np;
        z.alpha = m->co.qo;
        z.out = cs.tmp[c];
        z.ldout = np;
        z.ncols = np;
        z.region = ch.region;
        s2.add(z, np, m->regions[ch.region].nb);
        g2.add(cs.S[c] + blk * t, cs.tmp[c], cs.S[c] + blk * t, cs.sig[c], np, np, np, np, np,
               np, 1.0, 1.0, 1, 0, m->regions[ch.region].nb, m->regions[ch.region].nb);
        g2.set_last_lower();  // Sigma_tt is symmetric: lower tiles, then mirrored
        {
          InvTask mt{};
          mt.M = cs.sig[c];
          mt.np = np;
          mir.push_back(mt);
        }
        if (is_core(c, t)) {
          ExtractTask e{};
          e.M = cs.sig[c];
          e.ld = np;
          e.region = ch.region;
          e.t = ch.t0 + t;
          e.kind = 0;
          e.sign = 1.0;
          e.out_slot = slot_base[c] + t * 4 + 0;
          e2.add(e, (np + 255) / 256);
        }
      }
    }
    tak.stencil(m->arena, s1);
    tak.gemm(m->arena, g1);
    tak.extract(m->arena, e1);
    tak.stencil(m->arena, s2);
    tak.gemm(m->arena, g2);
    tak.mirror(m->arena, mir);
    tak.extract(m->arena, e2);
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
        pt.P = (t == 0) ? m->sub_y[c] : m->sub_pan[c][t];
        pt.region = ch.region;
        pt.t = ch.t0 + t;
        pt.t0 = ch.t0;
        pt.T = ch.T;
        pt.mode = 2;
        rt.add(pt, panel_tiles(np, nk), 16.0 * m->regions[ch.region].nb * nk);
      }
    }
    cor.panels(m->arena, rt, x, nullptr, nk);
    std::vector<int> stop(nchains);
    for (int c = 0; c < nchains; ++c) stop[c] = std::max(lc0(c) - 1, 0);
    build_solve(m, cs, m->sub_pan, m->sub_y, nk, stop, cor);
    TileList<McTask> mt;
    for (int c = 0; c < nchains; ++c) {
      const Chain& ch = cs.chains[c];
      for (int t = lc0(c); t <= lc1(c); ++t) {
        McTask k{};
        k.mu[0] = (t - 1 >= 0) ? m->sub_pan[c][t - 1] : nullptr;
        k.mu[1] = m->sub_pan[c][t];
        k.mu[2] = (t + 1 < ch.T) ? m->sub_pan[c][t + 1] : nullptr;
        k.np = cs.np[c];
        k.region = ch.region;
        k.t = ch.t0 + t;
        k.out_slot = slot_base[c] + t * 4 + 3;
        mt.add(k, cs.np[c] / 64);
      }
    }
    cor.mc(m->arena, mt, nk);
  }
  HIPCHK(m->arena.upload(s));
  RunCtx rc;
  rc.diag_out = diag_out;
  rc.partial = det_part;
  rc.nchunk_max = nchunk_max;
  st = run(m, tak, rc);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  double t2 = now_s();
  rc.partial = mc_part;
  rc.nchunk_max = mc_chunks;
  st = run(m, cor, rc);
  if (st != RBMC_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  double t3 = now_s();
  // ---- traces: combine partial sums with the temporal weights ----
  std::vector<double> hdet(det_len), hmc(mc_len);
  HIPCHK(hipMemcpy(hdet.data(), det_part, det_len * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hmc.data(), mc_part, mc_len * 8, hipMemcpyDeviceToHost));
  const Coefs& co = m->co;
  double tr[4] = {0, 0, 0, 0};
  double ratio_sum = 0.0;  // sum over nodes of (MC part) / (estimate)
  for (int c = 0; c < nchains; ++c) {
    const Chain& ch = cs.chains[c];
    for (int t = lc0(c); t <= lc1(c); ++t) {
      const int tg = ch.t0 + t;
      // deterministic: slot 0 (t,t), slot 1 (t,t+1), slot 2 (t,t-1)
      double Fd = 0, Fq[3] = {0, 0, 0}, Fk[3] = {0, 0, 0};
      for (int sl = 0; sl < 3; ++sl) {
        const int slot = slot_base[c] + t * 4 + sl;
        for (int ch2 = 0; ch2 < nchunk_max; ++ch2) {
          const double* pp = &hdet[((size_t)slot * nchunk_max + ch2) * 3];
          if (sl == 0) Fd += pp[0];
          Fq[sl] += pp[1];
          Fk[sl] += pp[2];
        }
      }
      // Monte Carlo: slot 3, components [t-1, t, t+1] for Q_s and K, then D
      double G[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (nk > 0) {
        const int slot = slot_base[c] + t * 4 + 3;
        for (int ch2 = 0; ch2 < mc_chunks; ++ch2)
          for (int j = 0; j < 8; ++j) G[j] += hmc[((size_t)slot * mc_chunks + ch2) * 8 + j];
      }
      ratio_sum += G[7];
      const double wq0 = co.qd[tg], wqo = co.qo, wd0 = co.dqd[tg], wdo = co.dqo;
      const bool hm = (t - 1 >= 0), hp = (t + 1 < ch.T);
      // Q_s-weighted sums over (t,t), (t,t+1), (t,t-1)
      const double q_tt = Fq[0] + G[1];
      const double q_tp = hp ? Fq[1] + G[2] : 0.0;
      const double q_tm = hm ? Fq[2] + G[0] : 0.0;
      const double k_tt = Fk[0] + G[4];
      const double k_tp = hp ? Fk[1] + G[5] : 0.0;
      const double k_tm = hm ? Fk[2] + G[3] : 0.0;
      tr[0] += wq0 * k_tt + wqo * (k_tp + k_tm);
      tr[1] += wq0 * q_tt + wqo * (q_tp + q_tm);
      tr[2] += wd0 * q_tt + wdo * (q_tp + q_tm);
      tr[3] += -2.0 * (Fd + G[6]);
    }
  }
  if (trace_out) {
    int j = 0;
    for (int b = 0; b < 4; ++b)
      if (o->grad_mask & (1u << b)) trace_out[j++] = tr[b];
  }
  if (rep) {
    // plug-in MC error: m_i ~ E[mu_i^2] chi2_{n_k} / n_k, so the mean absolute relative
    // error of the estimate is about sqrt(2/pi) sqrt(2/n_k) m_i / s2_i on average
    rep->err_estimate =
        nk > 0 ? std::sqrt(2.0 / M_PI) * std::sqrt(2.0 / nk) * ratio_sum / P.n : 0.0;
    rep->t_factor += t1 - t0;
    rep->t_takahashi = t2 - t1;
    rep->t_correct = t3 - t2;
    rep->peak_bytes = m->pool.bytes + m->work.bytes;
  }
  return RBMC_OK;
}

rbmc_status rbmc_sample(rbmc_model* m, const rbmc_est_opts* opts, const double* z, double* x,
                        rbmc_report* rep) {
  init_report(rep);
  if (!m || !z || !x) return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (opts->n_samples == 0) return RBMC_OK;
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  st = sample_impl(m, opts, z, x, rep);
  if (rep) rep->t_total = now_s() - t0;
  return st;
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
  st = estimate_impl(m, opts, x, diag_out, trace_out, rep);
  if (rep) rep->t_total = now_s() - t0;
  return st;
}

rbmc_status rbmc_estimate(rbmc_model* m, const rbmc_est_opts* opts, const double* z, uint64_t seed,
                          double* diag_out, double* trace_out, rbmc_report* rep) {
  (void)seed;
  init_report(rep);
  if (!m || !diag_out) return fail(RBMC_E_ARG, "NULL argument");
  rbmc_status st = check_opts(opts, true);
  if (st != RBMC_OK) return st;
  if (opts->n_samples > 0 && !z)
    return fail(RBMC_E_UNSUPPORTED, "z must be supplied (device sampling of z is not built)");
  if (opts->grad_mask && !trace_out) return fail(RBMC_E_ARG, "trace_out is NULL");
  HIPCHK(hipSetDevice(m->ctx->device));
  double t0 = now_s();
  rbmc_status st1 = RBMC_OK;
  if (opts->n_samples > 0) {
    st = ensure_work(m, opts->n_samples);
    if (st != RBMC_OK) return st;
    st1 = sample_impl(m, opts, z, m->w_x, rep);
    if (st1 < 0) return st1;
  }
  double ts = rep ? rep->t_sample : 0.0;
  int itmax = rep ? rep->pcg_it_max : 0;
  double itmean = rep ? rep->pcg_it_mean : 0.0, maxres = rep ? rep->max_rel_residual : 0.0;
  st = estimate_impl(m, opts, m->w_x, diag_out, trace_out, rep);
  if (rep) {
    rep->t_sample = ts;
    rep->pcg_it_max = itmax;
    rep->pcg_it_mean = itmean;
    rep->max_rel_residual = maxres;
    rep->t_total = now_s() - t0;
  }
  if (st != RBMC_OK) return st;
  return st1;
}

}  // extern "C"
