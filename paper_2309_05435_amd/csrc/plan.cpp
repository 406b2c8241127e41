// Decomposition planner and model coefficients (host side).
//
// Cores Omega_p are time slabs x spatial boxes.  The graph of Q = Q_t (x) Q_s
// + D is the strong product of the time path (Q_t tridiagonal) and the
// 13-point spatial graph of Q_s (|dx| + |dy| <= 2), so the Alg. 4 extension
// of a core by n_l rounds of graph neighbours is the product
//   Omega_p* = {t : d_time <= n_l} x {s : L1 distance to the box <= 2 n_l}
// and the separator S_p = N(Omega_p*) \ Omega_p* is the shell at n_l + 1.
// Every Omega_p* is therefore a block-tridiagonal chain of dense spatial
// blocks over one spatial region R_p, which is what the kernels factor.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "rbmc_impl.h"

namespace rbmc {

int piece_len(int k, int len, int parts) { return len / parts + (k < len % parts ? 1 : 0); }

int piece_start(int k, int len, int parts) {
  int base = len / parts, extra = len % parts;
  return k * base + std::min(k, extra);
}

static int find_region(Plan& plan, int x0, int x1, int y0, int y1, int hops) {
  for (int r = 0; r < (int)plan.regions.size(); ++r) {
    const Region& g = plan.regions[r];
    if (g.x0 == x0 && g.x1 == x1 && g.y0 == y0 && g.y1 == y1 && g.hops == hops) return r;
  }
  Region g;
  g.x0 = x0;
  g.x1 = x1;
  g.y0 = y0;
  g.y1 = y1;
  g.hops = hops;
  const int mx = plan.mx, my = plan.my;
  std::vector<int> loc((size_t)mx * my, -1);
  for (int iy = 0; iy < my; ++iy)
    for (int ix = 0; ix < mx; ++ix) {
      int dx = std::max(std::max(x0 - ix, ix - x1), 0);
      int dy = std::max(std::max(y0 - iy, iy - y1), 0);
      if (dx + dy <= 2 * hops) {
        loc[(size_t)iy * mx + ix] = (int)g.nodes.size();
        g.nodes.push_back(iy * mx + ix);
        g.in_box.push_back(dx == 0 && dy == 0);
      }
    }
  g.nbr.assign(g.nodes.size() * kNS, -1);
  for (size_t a = 0; a < g.nodes.size(); ++a) {
    int s = g.nodes[a], ix = s % mx, iy = s / mx;
    for (int k = 0; k < kNS; ++k) {
      int jx = ix + kSdx[k], jy = iy + kSdy[k];
      if (jx < 0 || jx >= mx || jy < 0 || jy >= my) continue;
      g.nbr[a * kNS + k] = loc[(size_t)jy * mx + jx];
    }
  }
  plan.regions.push_back(std::move(g));
  return (int)plan.regions.size() - 1;
}

std::string make_plan(const rbmc_model_desc& d, const rbmc_decomp_desc& dc, Plan& plan) {
  if (d.mx < 2 || d.my < 2 || d.T < 1) return "grid needs mx, my >= 2 and T >= 1";
  // the kernels index the nodes of one sample with 32-bit integers
  if ((long long)d.mx * d.my * d.T >= (1LL << 31)) return "mx my T must be below 2^31";
  if (dc.n_tslabs < 1 || dc.n_tslabs > d.T) return "n_tslabs must lie in [1, T]";
  if (dc.n_tiles_x < 1 || dc.n_tiles_x > d.mx) return "n_tiles_x must lie in [1, mx]";
  if (dc.n_tiles_y < 1 || dc.n_tiles_y > d.my) return "n_tiles_y must lie in [1, my]";
  if (dc.overlap_hops < 0) return "overlap_hops must be >= 0";
  if (dc.separators != 0 && dc.separators != 1) return "separators must be 0 or 1";
  if (dc.separators && dc.overlap_hops != 0) return "separators need overlap_hops = 0";
  plan = Plan();
  plan.mx = d.mx;
  plan.my = d.my;
  plan.T = d.T;
  plan.ns = d.mx * d.my;
  plan.n = plan.ns * d.T;
  plan.P = dc.n_tslabs;
  plan.ntx = dc.n_tiles_x;
  plan.nty = dc.n_tiles_y;
  plan.hops = dc.overlap_hops;
  for (int k = 0; k < plan.P; ++k) {
    plan.slab_t0.push_back(piece_start(k, d.T, plan.P));
    plan.slab_len.push_back(piece_len(k, d.T, plan.P));
  }
  for (int k = 0; k < plan.ntx; ++k) {
    plan.tile_x0.push_back(piece_start(k, d.mx, plan.ntx));
    plan.tile_xlen.push_back(piece_len(k, d.mx, plan.ntx));
  }
  for (int k = 0; k < plan.nty; ++k) {
    plan.tile_y0.push_back(piece_start(k, d.my, plan.nty));
    plan.tile_ylen.push_back(piece_len(k, d.my, plan.nty));
  }
  const int h = plan.hops;
  plan.sep = dc.separators;
  if (plan.sep) {  // Alg. 2: one step and two grid lines between neighbouring cores
    for (int k = 1; k < plan.P; ++k)
      if (plan.slab_len[k] < 2) return "separators need slabs of >= 2 steps";
    for (int k = 1; k < plan.ntx; ++k)
      if (plan.tile_xlen[k] < 3) return "separators need tiles of >= 3 lines";
    for (int k = 1; k < plan.nty; ++k)
      if (plan.tile_ylen[k] < 3) return "separators need tiles of >= 3 lines";
  }
  for (int sl = 0; sl < plan.P; ++sl)
    for (int ty = 0; ty < plan.nty; ++ty)
      for (int tx = 0; tx < plan.ntx; ++tx) {
        int p = (sl * plan.nty + ty) * plan.ntx + tx;
        int x0 = plan.tile_x0[tx], x1 = x0 + plan.tile_xlen[tx] - 1;
        int y0 = plan.tile_y0[ty], y1 = y0 + plan.tile_ylen[ty] - 1;
        int ct0 = plan.slab_t0[sl], cT = plan.slab_len[sl];
        if (dc.pc_tslabs <= 0) {  // block-Jacobi blocks: the whole slab x tile
          Chain b;
          b.region = find_region(plan, x0, x1, y0, y1, 0);
          b.t0 = ct0;
          b.T = cT;
          b.ct0 = ct0;
          b.cT = cT;
          b.core_id = p;
          plan.bj.push_back(b);
        }
        if (plan.sep) {
          if (tx > 0) x0 += 2;
          if (ty > 0) y0 += 2;
          if (sl > 0) {
            ++ct0;
            --cT;
          }
        }
        Chain c;
        c.region = find_region(plan, x0, x1, y0, y1, h);
        c.t0 = std::max(0, ct0 - h);
        c.T = std::min(d.T - 1, ct0 + cT - 1 + h) - c.t0 + 1;
        c.ct0 = ct0;
        c.cT = cT;
        c.core_id = p;
        plan.sub.push_back(c);
      }
  if (dc.pc_tslabs > 0) {
    const int pt = dc.pc_tslabs, px = dc.pc_tiles_x, py = dc.pc_tiles_y;
    if (pt > d.T || px < 1 || px > d.mx || py < 1 || py > d.my)
      return "preconditioner blocks: pc_tslabs in [1, T], pc_tiles_x in [1, mx], pc_tiles_y in [1, my]";
    for (int sl = 0; sl < pt; ++sl)
      for (int ty = 0; ty < py; ++ty)
        for (int tx = 0; tx < px; ++tx) {
          Chain b;
          const int x0 = piece_start(tx, d.mx, px), y0 = piece_start(ty, d.my, py);
          b.region = find_region(plan, x0, x0 + piece_len(tx, d.mx, px) - 1, y0,
                                 y0 + piece_len(ty, d.my, py) - 1, 0);
          b.t0 = piece_start(sl, d.T, pt);
          b.T = piece_len(sl, d.T, pt);
          b.ct0 = b.t0;
          b.cT = b.T;
          b.core_id = -1;
          plan.bj.push_back(b);
        }
  }
  if (plan.sep) {
    std::vector<int32_t> lab((size_t)plan.n);
    plan_labels(plan, lab.data());
    for (int i = 0; i < plan.n; ++i)
      if (lab[i] < 0) plan.sep_nodes.push_back(i);
  }
  return "";
}

// core of every node; -1 for the separator nodes of Alg. 2
void plan_labels(const Plan& plan, int32_t* label) {
  std::fill(label, label + plan.n, -1);
  for (const Chain& c : plan.sub) {
    const Region& g = plan.regions[c.region];
    for (int t = c.ct0; t < c.ct0 + c.cT; ++t)
      for (int a = 0; a < g.nb(); ++a)
        if (g.in_box[a]) label[(size_t)t * plan.ns + g.nodes[a]] = c.core_id;
  }
}

void plan_state(const Plan& plan, int p, uint8_t* state) {
  std::fill(state, state + plan.n, (uint8_t)0);
  const Chain& c = plan.sub[p];
  const Region& g = plan.regions[c.region];
  const int h = plan.hops;
  const int mx = plan.mx, my = plan.my;
  // distance of every node to the core in the strong product metric
  for (int t = 0; t < plan.T; ++t) {
    int dt = std::max(std::max(c.ct0 - t, t - (c.ct0 + c.cT - 1)), 0);
    if (dt > h + 1) continue;
    for (int iy = 0; iy < my; ++iy)
      for (int ix = 0; ix < mx; ++ix) {
        int dx = std::max(std::max(g.x0 - ix, ix - g.x1), 0);
        int dy = std::max(std::max(g.y0 - iy, iy - g.y1), 0);
        int ds = (dx + dy + 1) / 2;
        int dd = std::max(dt, ds);
        uint8_t v = 0;
        if (dd == 0)
          v = 1;
        else if (dd <= h)
          v = 2;
        else if (dd == h + 1)
          v = 3;
        state[(size_t)t * plan.ns + iy * mx + ix] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// Coefficients of Q_s, dQ_s/dlog kappa, F_s (per spatial node) and of Q_t,
// dQ_t/drho, L (per time step).
//   G: graph Laplacian of the 4-neighbour grid (G_ss = deg s, G_s,s+e = -1)
//   G^2: (s,s) deg^2 + deg; (s,s+e) -(deg s + deg s+e); (s,s+2e) 1;
//        (s, s+e1+e2) 2.
//   Q_s = tau (kappa^4 h^2 I + 2 kappa^2 G + G^2 / h^2)
//   K   = tau (4 kappa^4 h^2 I + 4 kappa^2 G)
//   F_s = sqrt(tau) (kappa^2 h^2 I + G) / h,   F_s F_s^T = Q_s
//   Q_t = R / (1 - rho^2), R = tridiag(-rho; 1, 1 + rho^2, ..., 1; -rho)
//   L: (L x)_0 = x_0, (L x)_t = (x_t - rho x_{t-1}) / sqrt(1 - rho^2),  Q_t = L^T L
// ---------------------------------------------------------------------------
void make_coefs(int mx, int my, int T, double h, double log_kappa, double log_tau, double rho,
                double log_sigma, Coefs& c) {
  const int ns = mx * my;
  c.kappa = std::exp(log_kappa);
  c.tau = std::exp(log_tau);
  c.rho = rho;
  c.sigma = std::exp(log_sigma);
  c.h = h;
  const double k2 = c.kappa * c.kappa, k4 = k2 * k2, h2 = h * h, tau = c.tau;
  auto inside = [&](int x, int y) { return x >= 0 && x < mx && y >= 0 && y < my; };
  auto deg = [&](int x, int y) {
    return (int)inside(x - 1, y) + (int)inside(x + 1, y) + (int)inside(x, y - 1) +
           (int)inside(x, y + 1);
  };
  c.qs.assign((size_t)kNS * ns, 0.0);
  c.kk.assign((size_t)kN5 * ns, 0.0);
  c.fs.assign((size_t)kN5 * ns, 0.0);
  const double sqt = std::sqrt(tau);
  for (int iy = 0; iy < my; ++iy)
    for (int ix = 0; ix < mx; ++ix) {
      const int s = iy * mx + ix;
      const int ds = deg(ix, iy);
      for (int k = 0; k < kNS; ++k) {
        int jx = ix + kSdx[k], jy = iy + kSdy[k];
        if (!inside(jx, jy)) continue;
        double g = 0.0, g2 = 0.0, id = 0.0;
        int l1 = std::abs(kSdx[k]) + std::abs(kSdy[k]);
        if (k == 0) {
          id = 1.0;
          g = ds;
          g2 = (double)ds * ds + ds;
        } else if (l1 == 1) {
          g = -1.0;
          g2 = -(double)(ds + deg(jx, jy));
        } else if (kSdx[k] == 0 || kSdy[k] == 0) {
          g2 = 1.0;
        } else {
          g2 = 2.0;
        }
        c.qs[(size_t)k * ns + s] = tau * (k4 * h2 * id + 2.0 * k2 * g + g2 / h2);
        if (k < kN5) {
          c.kk[(size_t)k * ns + s] = tau * (4.0 * k4 * h2 * id + 4.0 * k2 * g);
          c.fs[(size_t)k * ns + s] = sqt * (k2 * h2 * id + g) / h;
        }
      }
    }
  const double a = 1.0 - rho * rho;
  c.qd.assign(T, 0.0);
  c.dqd.assign(T, 0.0);
  c.ld.assign(T, 0.0);
  for (int t = 0; t < T; ++t) {
    bool end = (t == 0 || t == T - 1);
    double R = end ? 1.0 : 1.0 + rho * rho;
    double dR = end ? 0.0 : 2.0 * rho;
    c.qd[t] = (T == 1) ? 1.0 : R / a;
    c.dqd[t] = (T == 1) ? 0.0 : dR / a + 2.0 * rho * R / (a * a);
    c.ld[t] = (t == 0) ? 1.0 : 1.0 / std::sqrt(a);
  }
  c.qo = -rho / a;
  c.dqo = -1.0 / a - 2.0 * rho * rho / (a * a);
  c.lo = -rho / std::sqrt(a);
  c.dobs = 1.0 / (c.sigma * c.sigma);
}

}  // namespace rbmc
