// Test driver for the host bidiagonal SVD: reads "k nvec", then d (k values)
// and e (k-1 values) from stdin, and prints sigma, the last row of P, and the
// first nvec columns of Q and P, one value per line, or "FAIL".
#include <cstdio>
#include <vector>

#include "bidiag.h"

int main() {
  int k = 0, nvec = 0;
  if (std::scanf("%d %d", &k, &nvec) != 2 || k < 1) return 2;
  std::vector<double> d(k), e(k > 1 ? k - 1 : 0);
  for (double &x : d)
    if (std::scanf("%lf", &x) != 1) return 2;
  for (double &x : e)
    if (std::scanf("%lf", &x) != 1) return 2;
  svt::BidiagSVD out;
  if (!svt::bidiag_svd(d, e, out)) {
    std::printf("FAIL\n");
    return 0;
  }
  svt::bidiag_vectors(d, e, nvec, out);
  for (double x : out.sigma) std::printf("%.17e\n", x);
  for (double x : out.p_last) std::printf("%.17e\n", x);
  for (double x : out.Q) std::printf("%.17e\n", x);
  for (double x : out.P) std::printf("%.17e\n", x);
  return 0;
}
