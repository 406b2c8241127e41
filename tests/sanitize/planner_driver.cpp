// Host sanitizer driver for the decomposition planner and the model
// coefficients (the host code behind rbmc_plan_query and rbmc_model_create),
// test infrastructure.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer for the host; any report aborts the run.
#include <cstdio>
#include <vector>

#include "rbmc_impl.h"

using namespace rbmc;

int main() {
  const int cases[][7] = {{16, 16, 10, 4, 1, 1, 1}, {12, 10, 9, 3, 2, 2, 1},
                          {13, 13, 8, 2, 3, 2, 2},  {9, 9, 7, 7, 1, 1, 0},
                          {20, 17, 5, 1, 3, 4, 2},  {7, 7, 1, 1, 1, 1, 1},
                          {64, 48, 12, 3, 4, 3, 3}, {8, 8, 10, 11, 1, 1, 1}};
  int bad = 0;
  for (const auto& c : cases) {
    const int mx = c[0], my = c[1], T = c[2];
    const int n = mx * my * T;
    std::vector<unsigned char> mask(n);
    for (int i = 0; i < n; ++i) mask[i] = (i * 7919) % 10 < 3;
    rbmc_model_desc d{};
    d.mx = mx;
    d.my = my;
    d.T = T;
    d.h = 1.0 / (mx - 1);
    d.log_kappa = 2.0;
    d.rho = 0.9;
    d.obs_mask = mask.data();
    rbmc_decomp_desc dc{};
    dc.n_tslabs = c[3];
    dc.n_tiles_x = c[4];
    dc.n_tiles_y = c[5];
    dc.overlap_hops = c[6];
    Plan plan;
    const std::string e = make_plan(d, dc, plan);
    if (!e.empty()) {  // the last case is invalid on purpose (11 slabs of 10 steps)
      bad += (c[3] <= T);
      continue;
    }
    std::vector<int32_t> label(n);
    std::vector<uint8_t> state(n);
    plan_labels(plan, label.data());
    for (size_t p = 0; p < plan.sub.size(); ++p) plan_state(plan, (int)p, state.data());
    Coefs co;
    make_coefs(mx, my, T, d.h, d.log_kappa, d.log_tau, d.rho, d.log_sigma, co);
  }
  if (bad) {
    std::fprintf(stderr, "%d valid cases refused\n", bad);
    return 1;
  }
  std::printf("planner driver ok\n");
  return 0;
}
