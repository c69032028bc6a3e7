// Test driver for the library's host Hermitian eigensolvers: reads n and an n x n complex
// matrix (row-major, re im pairs, binary doubles) from stdin, writes the eigenvalues and
// the eigenvectors (columns of a row-major n x n matrix) of the method named in argv[1]
// ("tridiag" or "jacobi") to stdout in the same binary form.
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

#include "eigh_host.h"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  int n = 0;
  if (std::fread(&n, sizeof(int), 1, stdin) != 1 || n < 0) return 3;
  std::vector<std::complex<double>> A((size_t)n * n), Z;
  if (std::fread(A.data(), sizeof(double), 2 * (size_t)n * n, stdin) != 2 * (size_t)n * n) return 4;
  std::vector<double> w;
  const int r = std::strcmp(argv[1], "jacobi") == 0 ? eigh_jacobi(n, A, w, Z) : eigh_tridiag(n, A, w, Z);
  if (r < 0) return 5;
  std::fwrite(w.data(), sizeof(double), (size_t)n, stdout);
  std::fwrite(Z.data(), sizeof(double), 2 * (size_t)n * n, stdout);
  return 0;
}
