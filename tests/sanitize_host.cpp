// Host-side checker of the set-up code under AddressSanitizer and
// UndefinedBehaviorSanitizer: reads a mesh and problem description, runs the
// host set-up (side analysis, classes, Algorithm 1, coarse maps, coarse
// assembly), forces the nested-dissection ordering and factors K on the host,
// and prints the sizes.  Built and run by tests/test_host_sanitizers.py; no
// device code is involved.
//
// Input (stdin): x0 x1 y0 y1 base_nx base_ny n_leaves k l discard_tol l_per_edge
// then n_leaves lines "level ix iy degree eps_r".
#include <cstdio>
#include <vector>

#include "../paper_1808_04713_amd/csrc/internal.hpp"

namespace hdp {
[[noreturn]] void fail(hdp_status s, const std::string& msg) { throw Error{s, msg}; }
void check_hip(hipError_t, const char*) {}
}  // namespace hdp

int main() {
  double x0, x1, y0, y1, k, tau;
  int bnx, bny, nl, l, per_edge;
  if (std::scanf("%lf %lf %lf %lf %d %d %d %lf %d %lf %d", &x0, &x1, &y0, &y1, &bnx, &bny, &nl, &k, &l, &tau,
                 &per_edge) != 11)
    return 2;
  std::vector<int> leaf(3 * size_t(nl)), deg(nl);
  std::vector<double> eps(nl);
  for (int i = 0; i < nl; ++i)
    if (std::scanf("%d %d %d %d %lf", &leaf[3 * i], &leaf[3 * i + 1], &leaf[3 * i + 2], &deg[i], &eps[i]) != 5)
      return 2;
  hdp_mesh mesh{x0, x1, y0, y1, bnx, bny, nl, leaf.data(), deg.data()};
  hdp_problem prob{};
  prob.k = k;
  prob.eps_r = eps.data();
  prob.l = l;
  prob.discard_tol = tau;
  prob.l_per_edge = per_edge;
  try {
    hdp::Handle h;
    h.coarse_mode = 2;   // nested dissection whatever the size
    hdp::build_host(h, &mesh, &prob);
    std::vector<int64_t> kidx;
    std::vector<double2> kval;
    hdp::coarse_coo(h, kidx, kval);
    hdp::NDHost f;
    hdp::nd_factor(h, kidx, kval, f);
    std::printf("n_lambda %d n_coarse %d classes %zu factor_entries %zu band_bytes %.6e\n", h.nlam, h.nK,
                h.classes.size(), f.fac.size(), hdp::coarse_band_bytes(h.nK, kidx));
  } catch (const hdp::Error& e) {
    std::printf("error %d %s\n", int(e.status), e.msg.c_str());
    return 3;
  }
  return 0;
}
