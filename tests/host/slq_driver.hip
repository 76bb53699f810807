// Host driver for the tridiagonal eigensolver of the SLQ kernel (compiled by
// tests/test_slq_host.py).  Reads "n", the n diagonal and n-1 off-diagonal entries per case from
// stdin; prints "n fail" and then one line "lambda_i w_i" per eigenvalue, w_i being the square of
// the first component of its unit eigenvector.  Arrays are strided (as in the kernels) and hold
// n + 1 entries each, exactly as many as the kernels provide.
#include <cstdio>
#include <vector>

#include "../../paper_2310_00420_amd/csrc/k_slq.hip"

int main() {
  int n;
  const long stride = 3;
  while (std::scanf("%d", &n) == 1) {
    std::vector<double> dg((n + 1) * stride), of((n + 1) * stride), zz((n + 1) * stride);
    for (int i = 0; i < n; ++i) std::scanf("%lf", &dg[i * stride]);
    for (int i = 0; i < n - 1; ++i) std::scanf("%lf", &of[i * stride]);
    for (int i = 0; i < n; ++i) zz[i * stride] = i == 0 ? 1.0 : 0.0;
    const int f = cmtcs::tridiag_eig_first_row<long>(dg.data(), of.data(), zz.data(), n, stride,
                                                     30 * n, cmtcs::RsqHost());
    std::printf("%d %d\n", n, f);
    for (int i = 0; i < n; ++i)
      std::printf("%.17g %.17g\n", dg[i * stride], zz[i * stride] * zz[i * stride]);
  }
  return 0;
}
