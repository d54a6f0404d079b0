// Test driver for the host dense kernels of the randomised partial SVD:
// reads "op rows cols" and a column-major matrix from stdin.  op 0: prints
// the orthonormal basis of orth_columns; op 1: prints sigma, Vw and Uw of
// jacobi_svd_tall (or "FAIL").  One value per line.
#include <cstdio>
#include <vector>

#include "dense_host.h"

int main() {
  int op = 0, cols = 0;
  long long rows = 0;
  if (std::scanf("%d %lld %d", &op, &rows, &cols) != 3 || rows < 1 || cols < 1) return 2;
  std::vector<double> Z((size_t)rows * cols);
  for (double &x : Z)
    if (std::scanf("%lf", &x) != 1) return 2;
  if (op == 0) {
    svt::orth_columns(Z.data(), rows, cols);
    for (double x : Z) std::printf("%.17e\n", x);
    return 0;
  }
  std::vector<double> s, V, U;
  if (!svt::jacobi_svd_tall(Z.data(), rows, cols, s, V, U)) {
    std::printf("FAIL\n");
    return 0;
  }
  for (double x : s) std::printf("%.17e\n", x);
  for (double x : V) std::printf("%.17e\n", x);
  for (double x : U) std::printf("%.17e\n", x);
  return 0;
}
