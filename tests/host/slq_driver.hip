// Host driver for the log-determinant quadrature of the SLQ kernel (compiled by
// tests/test_slq_host.py).  Per case, reads from stdin "n", the n diagonal and n-1 off-diagonal
// entries of a symmetric tridiagonal, then "m" and m shifts x.  Prints "n pd lambda_min
// lambda_max logq" (logq = e_1^T log(T) e_1, 0 unless pd) and a line with the m Sturm counts
// (eigenvalues below x).  The per-lane routines are the kernel's own; the wave's lanes are
// emulated by loops in the kernel's order of rounds and points.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2310_00420_amd/csrc/k_slq.hip"

using namespace cmtcs;

int main() {
  int n;
  while (std::scanf("%d", &n) == 1) {
    std::vector<TriRow> r(n);
    std::vector<double> e(n > 1 ? n - 1 : 0);
    for (int i = 0; i < n; ++i) std::scanf("%lf", &r[i].a);
    for (int i = 0; i < n - 1; ++i) std::scanf("%lf", &e[i]);
    for (int i = 0; i < n; ++i) r[i].b2 = i + 1 < n ? e[i] * e[i] : 0.0;
    int m;
    std::scanf("%d", &m);
    std::vector<double> xs(m);
    for (int i = 0; i < m; ++i) std::scanf("%lf", &xs[i]);
    double glo = INFINITY, ghi = -INFINITY;
    for (int i = 0; i < n; ++i) {
      const double bl = i > 0 ? std::fabs(e[i - 1]) : 0.0;
      const double bu = i + 1 < n ? std::fabs(e[i]) : 0.0;
      glo = std::fmin(glo, r[i].a - bl - bu);
      ghi = std::fmax(ghi, r[i].a + bl + bu);
    }
    sec_start(glo, ghi);
    double lo[2] = {glo, glo}, hi[2] = {ghi, ghi};
    for (int it = 0; it < kSecRounds; ++it)
      for (int end = 0; end < 2; ++end) {
        uint32_t hit = 0;
        for (int k = 1; k <= kSecPoints; ++k)
          if (sturm_count(r.data(), n, sec_point(lo[end], hi[end], k), ScaleHost()) >=
              (end ? n : 1))
            hit |= 1u << (k - 1);
        sec_update(lo[end], hi[end], hit);
      }
    const bool pd = lo[0] > 0.0;
    double acc = 0.0;
    if (pd) {
      double s0;
      int nodes;
      quad_range(lo[0], hi[1], s0, nodes);
      for (int j = 0; j < nodes; ++j) acc += quad_node(r.data(), n, s0 + j * kQuadStep, ScaleHost());
      acc *= kQuadStep;
    }
    std::printf("%d %d %.17g %.17g %.17g\n", n, pd ? 1 : 0, 0.5 * (lo[0] + hi[0]),
                0.5 * (lo[1] + hi[1]), acc);
    for (int i = 0; i < m; ++i)
      std::printf("%d%c", sturm_count(r.data(), n, xs[i], ScaleHost()), i + 1 < m ? ' ' : '\n');
    if (m == 0) std::printf("\n");
  }
  return 0;
}
